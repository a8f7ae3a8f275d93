"""Serving loop: continuous batching with admission by tableau bytes.

Each request's outcome bytes must be identical when served alone and when
served in a mix of overlapping requests (tolerance 0), and agree with the CPU
oracle on a small subset."""
import numpy as np
import pytest
import torch

import oracle
from inputs import serving_workload

pytestmark = pytest.mark.gpu


def _workload(count=20, rate=400.0, n_hi=384, shots_hi=200, seed=4):
    reqs = serving_workload(count, rate, seed=seed, n_hi=n_hi, shots_hi=shots_hi)
    return [r.circuit for r in reqs], [r.arrival for r in reqs]


def test_mix_equals_alone_and_oracle():
    from paper_2408_00384_amd.serving import Server, summarize
    circs, arr = _workload()
    srv = Server(budget_bytes=256 << 20, lanes=4)
    alone = srv.run(circs, arr, realtime=False, one_at_a_time=True)
    alone_out = {i: r.outcomes.copy() for i, r in alone.items()}
    mix = srv.run(circs, arr, realtime=True)
    st = summarize(mix)
    assert st["completed"] == len(circs)
    for i in range(len(circs)):
        assert np.array_equal(alone_out[i], mix[i].outcomes), "request %d differs in the mix" % i
    # small ones against the oracle (every shot)
    for i, c in enumerate(circs):
        if c.n <= 48:
            for s in range(c.shots):
                ref, _ = oracle.run_shot(c, s)
                assert np.array_equal(mix[i].outcomes[s], ref), (i, s)
    assert set(st["paths"]) == {"hbm", "batch"}
    srv.close()


def test_admission_respects_budget_and_rejects_oversized():
    from paper_2408_00384_amd import cliff_tab_bytes
    from paper_2408_00384_amd.serving import Server, batch_request_bytes
    circs, arr = _workload(count=12, rate=1e6, n_hi=300, shots_hi=150, seed=9)
    # what a request holds: its tableau on an HBM lane, its op stream and
    # outcomes on the batch lane
    biggest = max(max(cliff_tab_bytes(c.n, c.shots), batch_request_bytes(c)) for c in circs)
    budget = 2 * biggest + 4096
    srv = Server(budget_bytes=budget, lanes=6)
    res = srv.run(circs, arr, realtime=False)
    assert all(r.error is None for r in res.values())
    assert srv.alloc.peak <= srv.alloc.size
    assert srv.alloc.used == 0
    # a request larger than the whole budget is rejected, the rest still served
    from inputs import layered_circuit
    big = layered_circuit(4096, 2, 1024, gen_seed=1)
    assert cliff_tab_bytes(big.n, big.shots) > budget
    res = srv.run(circs[:3] + [big], arr[:3] + [0.0], realtime=False)
    assert res[3].error is not None
    assert all(res[i].error is None and res[i].outcomes is not None for i in range(3))
    srv.close()


def test_large_requests_in_a_mix_vs_stored_oracle():
    """Three requests of the 96-request serving workload with n between 1,000
    and 1,800 (depth 2n, 377 to 754 shots), served in a mix with small
    requests: the first 48 outcomes of shot 0, of a middle shot and of the
    last shot, and the random flags, against the oracle's stored prefixes."""
    import json
    import os
    import sys
    from inputs import serving_params, serving_request
    from paper_2408_00384_amd.serving import Server
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, golden)
    from make_golden import SERVING_COUNT
    rec = json.load(open(os.path.join(golden, "serving_prefix.json")))
    k = rec["prefix"]
    arrivals, ns, shots = serving_params(SERVING_COUNT, 1.0, seed=4)
    big = [serving_request(int(i), arrivals, ns, shots, seed=4).circuit for i in rec["requests"]]
    small, small_arr = _workload(count=8, rate=800.0, n_hi=200, shots_hi=60, seed=11)
    circs = big + small
    arr = [0.0, 0.001, 0.002] + [0.0005 * (j + 1) for j in range(len(small))]
    srv = Server(budget_bytes=4 << 30, lanes=4)
    res = srv.run(circs, arr, realtime=True)
    srv.close()
    for j, (i, v) in enumerate(rec["requests"].items()):
        c, r = big[j], res[j]
        assert r.error is None and r.path == "hbm"
        assert (c.n, c.shots) == (v["n"], v["shots"])
        want_kinds = np.unpackbits(np.frombuffer(bytes.fromhex(v["random"]), np.uint8), bitorder="little")[:k]
        assert np.array_equal(r.random[:k], want_kinds), "request %s random flags" % i
        for s, hx in v["outcomes"].items():
            want = np.unpackbits(np.frombuffer(bytes.fromhex(hx), np.uint8), bitorder="little")[:k]
            assert np.array_equal(r.outcomes[int(s), :k], want), "request %s shot %s" % (i, s)

"""GPU parity on uniformly random Clifford circuits (gates only: the paper's
Fig. 2a workload), single-tableau paths and the many-tableau launch, against
the oracle bit for bit (x, z and every sign column)."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from inputs import random_clifford

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ctx():
    from paper_2408_00384_amd import Context
    c = Context(0)
    yield c
    c.close()


def _tab(ctx, n, shots=1):
    from paper_2408_00384_amd import DeviceTableau
    return DeviceTableau(ctx, n, shots)


def _ref(c):
    return oracle.Tableau(c.n).apply_gates(c.ops, c.a, c.b).get()


def _assert_equal(gpu, ref):
    gx, gz, gr = gpu
    x, z, r = ref
    assert np.array_equal(gx, x), "x bits differ"
    assert np.array_equal(gz, z), "z bits differ"
    for s in range(gr.shape[0]):
        assert np.array_equal(gr[s], r), "signs differ (shot %d)" % s


def _digest(x, z, r):
    h = hashlib.sha256()
    for a in (x, z, r):
        h.update(np.ascontiguousarray(a, np.uint8).tobytes())
    return h.hexdigest()


@pytest.fixture(params=["per_layer", "fused"])
def gate_mode(request, ctx):
    from paper_2408_00384_amd import (GATES_AUTO, GATES_FUSED, GATES_PER_LAYER,
                                      cliff_ctx_set_gate_mode)
    cliff_ctx_set_gate_mode(ctx.handle, GATES_PER_LAYER if request.param == "per_layer" else GATES_FUSED)
    yield request.param
    cliff_ctx_set_gate_mode(ctx.handle, GATES_AUTO)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 64, 100, 257])
def test_random_clifford_single_tableau(ctx, gate_mode, n):
    c = random_clifford(n, [6, n])
    t = _tab(ctx, n, 2).apply_gates(c.ops, c.a, c.b)
    _assert_equal(t.export(), _ref(c))


@pytest.mark.parametrize("rows", [0, 32, 64, 128])
def test_many_tableaux_from_gate_lists(ctx, rows):
    """Mixed sizes in one launch (ragged row groups: groups past a tableau's
    2n rows exit), two shots each."""
    from paper_2408_00384_amd import cliff_apply_gates_many
    ns = [1, 2, 7, 33, 64, 65, 130, 257, 500]
    cs = [random_clifford(n, [7, n, j]) for j, n in enumerate(ns)]
    tabs = [_tab(ctx, c.n, 2) for c in cs]
    cliff_apply_gates_many([t.handle for t in tabs], [(c.ops, c.a, c.b) for c in cs], rows)
    for t, c in zip(tabs, cs):
        _assert_equal(t.export(), _ref(c))


def test_many_tableaux_device_resident_streams_twice(ctx):
    """Encoded streams resident in device memory, applied twice (the second
    launch starts from the first one's tableaux and pending sign flips)."""
    import torch
    from paper_2408_00384_amd import cliff_apply_encoded_many, cliff_encode_gates
    cs = [random_clifford(200, [8, j]) for j in range(8)]
    enc = [cliff_encode_gates(c.n, c.ops, c.a, c.b) for c in cs]
    dev = [torch.from_numpy(w.view(np.int64)).to("cuda:0") for w, _ in enc]
    torch.cuda.synchronize()
    tabs = [_tab(ctx, c.n) for c in cs]
    for _ in range(2):
        cliff_apply_encoded_many([t.handle for t in tabs], [d.data_ptr() for d in dev], [o for _, o in enc])
    for t, c in zip(tabs, cs):
        ref = oracle.Tableau(c.n).apply_gates(c.ops, c.a, c.b).apply_gates(c.ops, c.a, c.b).get()
        _assert_equal(t.export(), ref)


@pytest.mark.parametrize("n", [200, 500, 1000])
def test_vs_stored_oracle(ctx, n):
    """Four uniformly random Clifford circuits of n = 200, 500 or 1,000 qubits
    (about 10^6 gates each at n = 1,000) in one many-tableau launch, and
    circuit 0 through the single-tableau path, against the oracle's stored
    tableau digests."""
    from paper_2408_00384_amd import cliff_apply_gates_many
    rec = json.load(open(os.path.join(GOLDEN, "clifford_n%d.json" % n)))
    n = rec["n"]
    cs = [random_clifford(n, [5, n, int(i)]) for i in sorted(rec["circuits"], key=int)]
    for c, (i, v) in zip(cs, sorted(rec["circuits"].items(), key=lambda kv: int(kv[0]))):
        assert c.gate_count() == v["gates"]
    tabs = [_tab(ctx, n) for _ in cs]
    cliff_apply_gates_many([t.handle for t in tabs], [(c.ops, c.a, c.b) for c in cs])
    for t, (i, v) in zip(tabs, sorted(rec["circuits"].items(), key=lambda kv: int(kv[0]))):
        x, z, r = t.export()
        assert _digest(x, z, r[0]) == v["tableau_sha256"], "circuit %s" % i
    single = _tab(ctx, n).apply_gates(cs[0].ops, cs[0].a, cs[0].b)
    x, z, r = single.export()
    assert _digest(x, z, r[0]) == rec["circuits"]["0"]["tableau_sha256"]


def test_many_tableaux_errors(ctx):
    from paper_2408_00384_amd import CLIFF_EINVAL, CliffError, cliff_apply_gates_many
    c = random_clifford(5, [9])
    t = _tab(ctx, 5)
    u = _tab(ctx, 5)
    lst = (c.ops, c.a, c.b)
    for tabs, lists, rows in [([t.handle, t.handle], [lst, lst], 0),     # repeated tableau
                              ([t.handle], [lst], 48),                      # bad group size
                              ([t.handle], [(np.array([9], np.uint8), np.array([0], np.uint32),
                                             np.array([0], np.uint32))], 0)]:   # bad op
        with pytest.raises(CliffError) as e:
            cliff_apply_gates_many(tabs, lists, rows)
        assert e.value.code == CLIFF_EINVAL
    big = _tab(ctx, 10177)
    with pytest.raises(CliffError) as e:
        cliff_apply_gates_many([big.handle], [lst], 64)    # 2 n 8 bytes > LDS at 64 rows
    assert e.value.code == CLIFF_EINVAL
    mid = _tab(ctx, 5089)
    with pytest.raises(CliffError) as e:
        cliff_apply_gates_many([mid.handle], [lst], 128)   # 2 n 16 bytes > LDS at 128 rows
    assert e.value.code == CLIFF_EINVAL
    # nothing ran: both tableaux still |0...0>
    cliff_apply_gates_many([t.handle, u.handle], [lst, lst])
    for tab in (t, u):
        _assert_equal(tab.export(), _ref(c))

"""Write stored expected values for the large parity cases, from the oracle only.

    python tests/golden/make_golden.py mid      # n = 1,024: all 128 shots (~5 min on 8 cores)
    python tests/golden/make_golden.py shots1024 # n = 2,100, 1,024 shots: 18 sampled shots (~5 min)
    python tests/golden/make_golden.py serving  # three n >= 1,000 serving requests: prefixes (~2 min)
    python tests/golden/make_golden.py large    # n = 10,000, 1 shot (hours)
    python tests/golden/make_golden.py clifford [n ...] # uniform random Cliffords (n = 1,000: ~40 s)
    python tests/golden/make_golden.py xlarge   # n = 25,000: first 32 measurements (~3 min, 2.5 GB)

Values are the CPU oracle's results on the seeded circuits of ``inputs``;
nothing here touches the GPU library.  Tableau digests are SHA-256 over the
byte-per-bit arrays x (2n x n), z (2n x n) and r (2n), concatenated in that order.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from inputs import (layered_circuit, plain_large, plain_mid, plain_xlarge, random_clifford,  # noqa: E402
                    serving_params, serving_request)

WORKERS = max(1, min(8, os.cpu_count() or 1))

HERE = os.path.dirname(os.path.abspath(__file__))


def digest(x, z, r) -> str:
    h = hashlib.sha256()
    for a in (x, z, r):
        h.update(np.ascontiguousarray(a, np.uint8).tobytes())
    return h.hexdigest()


def bits_hex(bits) -> str:
    return np.packbits(np.asarray(bits, np.uint8), bitorder="little").tobytes().hex()


def _shot_record(args):
    c, s = args
    out, kind, (x, z, r) = oracle.run_shot(c, s, want_tableau=True)
    return s, {"outcomes": bits_hex(out), "random": bits_hex(kind), "tableau_sha256": digest(x, z, r)}


def _shots_parallel(c, shots):
    """Oracle records of the given shots, one process per shot (each shot is
    an independent oracle run: gates, then measure-all)."""
    import multiprocessing as mp
    with mp.get_context("fork").Pool(WORKERS) as pool:
        recs = dict(pool.imap_unordered(_shot_record, [(c, s) for s in shots]))
    return {str(s): recs[s] for s in sorted(recs)}


def make_mid():
    c = plain_mid()
    rec = {"workload": "n=1024, 100 layers, measure all, 128 shots (generator seed 1)",
           "seed": c.seed, "shots": _shots_parallel(c, range(c.shots))}
    t = oracle.Tableau(c.n).apply_circuit_gates(c)
    rec["after_gates_sha256"] = digest(*t.get())
    with open(os.path.join(HERE, "plain_mid.json"), "w") as f:
        json.dump(rec, f, indent=1)


def shots1024_circuit():
    """n = 2,100 (66 row words), 10 layers, measure all, 1,024 shots."""
    return layered_circuit(2100, 10, 1024, gen_seed=[70, 2100], circuit_id=70)


def shots1024_sample():
    """Shot 0, one shot inside every further 64-shot sign word (a different
    bit position in each), and the last shot, 1,023."""
    return [0] + [64 * j + (37 * j) % 64 for j in range(1, 16)] + [1023]


def make_shots1024():
    c = shots1024_circuit()
    rec = {"workload": "n=2100, 10 layers (generator seed [70, 2100]), measure all, 1024 shots",
           "seed": c.seed, "circuit_id": c.circuit_id,
           "shots": _shots_parallel(c, shots1024_sample())}
    with open(os.path.join(HERE, "shots1024_n2100.json"), "w") as f:
        json.dump(rec, f, indent=1)


# the serving workload: 96 requests (request i from generator seed [4, 2, i])
SERVING_COUNT = 96
SERVING_PREFIX = 48


def serving_golden_requests(lo=1000, hi=1800, count=3):
    """Indices of the first `count` requests of the 96-request serving
    workload with lo <= n <= hi."""
    _, ns, _ = serving_params(SERVING_COUNT, 1.0, seed=4)
    return [int(i) for i in np.flatnonzero((ns >= lo) & (ns <= hi))[:count]]


def _serving_record(args):
    i, shot_list = args
    arrivals, ns, shots = serving_params(SERVING_COUNT, 1.0, seed=4)
    c = serving_request(i, arrivals, ns, shots, seed=4).circuit
    t = oracle.Tableau(c.n).apply_circuit_gates(c)
    q = c.qubits[:SERVING_PREFIX]
    res = {}
    for s in shot_list:
        out, kind = t.clone().measure_list(q, seed=c.seed, circuit=c.circuit_id, shot=s)
        res[str(s)] = bits_hex(out)
    return i, {"n": c.n, "shots": c.shots, "random": bits_hex(kind), "outcomes": res}


def make_serving():
    _, ns, shots = serving_params(SERVING_COUNT, 1.0, seed=4)
    idx = serving_golden_requests()
    jobs = [(i, sorted({0, int(shots[i]) // 2, int(shots[i]) - 1})) for i in idx]
    import multiprocessing as mp
    with mp.get_context("fork").Pool(WORKERS) as pool:
        recs = dict(pool.imap_unordered(_serving_record, jobs))
    rec = {"workload": "serving requests i of the %d-request workload (seed 4) with 1000 <= n <= 1800: "
                       "gates (depth 2n), then the first %d measurements of the listed shots"
                       % (SERVING_COUNT, SERVING_PREFIX),
           "prefix": SERVING_PREFIX, "requests": {str(i): recs[i] for i in idx}}
    with open(os.path.join(HERE, "serving_prefix.json"), "w") as f:
        json.dump(rec, f, indent=1)


def make_large(checkpoint_every=16):
    c = plain_large()
    t0 = time.time()
    t = oracle.Tableau(c.n).apply_circuit_gates(c)
    rec = {"workload": "n=10000, 20 layers, measure all, 1 shot (generator seed 2)",
           "seed": c.seed, "after_gates_sha256": digest(*t.get()),
           "prefix_sha256": {}}
    print("gates done in %.1fs" % (time.time() - t0), flush=True)
    out = np.zeros(c.n, np.uint8)
    kind = np.zeros(c.n, np.uint8)
    for m in range(c.n):
        o, k = t.measure(int(c.qubits[m]), seed=c.seed, circuit=c.circuit_id, shot=0, m=m)
        out[m], kind[m] = o, k
        if (m + 1) in (1, 2, 4, 8, checkpoint_every, 64, 256):
            rec["prefix_sha256"][str(m + 1)] = digest(*t.get())
        if (m + 1) % 200 == 0:
            print("measured %d in %.1fs" % (m + 1, time.time() - t0), flush=True)
    rec["outcomes"] = bits_hex(out)
    rec["random"] = bits_hex(kind)
    rec["final_sha256"] = digest(*t.get())
    rec["anomalies"] = t.anomalies
    rec["oracle_seconds"] = time.time() - t0
    with open(os.path.join(HERE, "plain_large.json"), "w") as f:
        json.dump(rec, f, indent=1)


def make_clifford(n=1000, count=4, seed=5):
    """Tableaux after the gates of uniform random Clifford circuits i < count
    (generator seed [seed, n, i]) applied to |0...0>."""
    rec = {"workload": "uniform random Clifford circuits, n=%d, gates only (generator seed [%d, n, i])"
           % (n, seed), "n": n, "circuits": {}}
    for i in range(count):
        c = random_clifford(n, [seed, n, i], circuit_id=i)
        t0 = time.time()
        t = oracle.Tableau(n).apply_gates(c.ops, c.a, c.b)
        rec["circuits"][str(i)] = {"gates": c.gate_count(), "tableau_sha256": digest(*t.get()),
                                   "oracle_seconds": round(time.time() - t0, 2)}
        print("clifford", i, c.gate_count(), "gates", flush=True)
    with open(os.path.join(HERE, "clifford_n%d.json" % n), "w") as f:
        json.dump(rec, f, indent=1)


def make_xlarge(k=32):
    """Outcomes and random flags of the first k measurements (qubits 0..k-1,
    m = position, shot 0) after the gates of the n = 25,000 circuit."""
    c = plain_xlarge()
    t0 = time.time()
    t = oracle.Tableau(c.n).apply_circuit_gates(c)
    print("gates done in %.1fs" % (time.time() - t0), flush=True)
    out, kind = t.measure_list(np.arange(k), seed=c.seed, circuit=c.circuit_id, shot=0)
    rec = {"workload": "n=25000, 20 layers, 1 shot (generator seed 6), qubits 0..%d measured" % (k - 1),
           "seed": c.seed, "k": k, "outcomes": bits_hex(out), "random": bits_hex(kind),
           "anomalies": t.anomalies, "oracle_seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "plain_xlarge_prefix.json"), "w") as f:
        json.dump(rec, f, indent=1)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "mid"
    if what == "mid":
        make_mid()
    elif what == "shots1024":
        make_shots1024()
    elif what == "serving":
        make_serving()
    elif what == "large":
        make_large()
    elif what == "clifford":
        for n in (sys.argv[2:] or ["1000"]):
            make_clifford(n=int(n))
    elif what == "xlarge":
        make_xlarge()
    else:
        raise SystemExit("usage: make_golden.py mid|shots1024|serving|large|clifford|xlarge")

"""Write stored expected values for the large parity cases, from the oracle only.

    python tests/golden/make_golden.py mid      # n = 1,024: a few shots (~1 min)
    python tests/golden/make_golden.py large    # n = 10,000, 1 shot (hours)
    python tests/golden/make_golden.py clifford # n = 1,000 uniform random Cliffords (~40 s)
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
from inputs import plain_large, plain_mid, plain_xlarge, random_clifford  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def digest(x, z, r) -> str:
    h = hashlib.sha256()
    for a in (x, z, r):
        h.update(np.ascontiguousarray(a, np.uint8).tobytes())
    return h.hexdigest()


def bits_hex(bits) -> str:
    return np.packbits(np.asarray(bits, np.uint8), bitorder="little").tobytes().hex()


def make_mid(shots=(0, 1, 63, 127)):
    c = plain_mid()
    rec = {"workload": "n=1024, 100 layers, measure all, 128 shots (generator seed 1)",
           "seed": c.seed, "shots": {}}
    for s in shots:
        out, kind, (x, z, r) = oracle.run_shot(c, s, want_tableau=True)
        rec["shots"][str(s)] = {"outcomes": bits_hex(out), "random": bits_hex(kind),
                                "tableau_sha256": digest(x, z, r)}
        print("mid shot", s, "random", int(kind.sum()), flush=True)
    t = oracle.Tableau(c.n).apply_circuit_gates(c)
    rec["after_gates_sha256"] = digest(*t.get())
    with open(os.path.join(HERE, "plain_mid.json"), "w") as f:
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
    elif what == "large":
        make_large()
    elif what == "clifford":
        make_clifford()
    elif what == "xlarge":
        make_xlarge()
    else:
        raise SystemExit("usage: make_golden.py mid|large|clifford|xlarge")

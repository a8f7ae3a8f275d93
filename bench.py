#!/usr/bin/env python3
"""Benchmark of the stabilizer-tableau hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload large|mid|small]

A step runs one whole circuit of the workload through the C ABI: |0...0>
init, every gate layer (op stream already resident in HBM), then
Z-measurement of all qubits for all shots, outcomes copied back to the host.
Default workload: n = 10,000 qubits, 20 layers of random H/S/CNOT-matching,
measure all, 1 shot (the rowsum-dominated single-tableau case).

One JSON line is printed with circuits/s, the roofline of the dominant kernel
and the CPU oracle timed on a bounded sample of the same workload.  At the
default size the dominant kernel is k_blk, the blocked measurement pass
(random measurements applied 32 at a time as one low-rank update to the
tableau held in registers); where it does not run, the register-resident
rowsum kernel k_meas_xz.  Both keep the tableau on chip, so their bound is
the ALU: the method's algorithmic 32-bit lane operations (from the
device-side support counters) over the kernel's time (HIP events recorded on
its stream around every launch of the timed steps), against the MI355X's
vector rate.  The HBM-equivalent rate of the same work is kept as
effective_alg_gbs.  On the per-measurement path (n > 10,240) the sweep
streams the tableau through HBM and is reported against HBM.

Further legs on the same line: the n = 64 and n = 1,024 workloads, the
batched 4,096-circuit workload (batched vs one circuit per launch, wall and
kernel-only), the serving workload, the paper's Fig. 2a sweep of uniformly
random Cliffords over n, and the n = 25,000 HBM-bound sweep.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak
LDS_PEAK_GBS = 256 * 128 * 2.4   # 256 CUs x 128 B/clk x 2.4 GHz = 78,643 GB/s
# MI355X vector ALU: 157.3 TFLOP/s fp32 counts a fused multiply-add as two
# operations, so the chip retires 78.6e12 32-bit lane operations per second
VALU_PEAK_TOPS = 157.3 / 2

# HBM bytes per launch of the dominant kernel from hardware counters
# (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a copy of known
# size), valid only for the kernel sources they were taken on.
TRAFFIC = {
    "k_blk": {
        "sources": ("paper_2408_00384_amd/csrc/measure_block.hip", "paper_2408_00384_amd/csrc/internal.h"),
        "sha256": "c6b91930278990bdaec921c5e613334314a5fd1f9e98758708a7a49e753da28e",
        "bytes_per_launch": 2.504e+08,
        "summary": "profiles/k_blk_plain_n10000_measure_all.md",
    },
    "k_meas_xz": {
        "sources": ("paper_2408_00384_amd/csrc/measure_persist.hip", "paper_2408_00384_amd/csrc/internal.h"),
        "sha256": "09f7ac8514d610188a899c7140616b3bf5c1c5c6c1be21e5187d6928cdeecbf2",
        "bytes_per_launch": 1.1221e+09,
        "summary": "profiles/k_meas_xz_plain_n10000_measure_all.md",
    },
}


def traffic_for(kernel: str):
    import hashlib
    rec = TRAFFIC.get(kernel)
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return rec["bytes_per_launch"] if h.hexdigest() == rec["sha256"] else None

WORKLOADS = {
    "small": dict(desc="plain CHP n=64, 64 layers, measure all, 16 shots", steps=20, warmup=3),
    "mid": dict(desc="plain CHP n=1024, 100 layers, measure all, 128 shots", steps=5, warmup=1),
    "large": dict(desc="plain CHP n=10000, 20 layers, measure all, 1 shot", steps=3, warmup=1),
}


def alu_roofline(counters, n, steps, sweep_ms, launches, traffic, blocked=False):
    """Roofline of the register-resident kernel that measured (k_blk, the
    blocked pass, or k_meas_xz, one rowsum sweep per measurement).

    Per random measurement with pivot-row support s (columns where the pivot
    row is not I), s_x (with an X part) and s_z (with a Z part), the sweep
    does per 64-bit row word of a supported column: the anticommuting rows
    (1 op, 2 for Y), the -1 rows (1), the mod-4 counter (3) and the updates of
    the planes the pivot row touches (1 each): 4 s + 2 (s_x + s_z) word
    operations, i.e. 8 s + 4 (s_x + s_z) = 4 (2 s + s_x + s_z) 32-bit lane
    operations per row word.  The device counters give sum(2 s + s_x + s_z)
    through the algorithmic bytes (8 W (2 s + s_x + s_z + 3) + 80 n per random
    measurement, 8 n W per deterministic one).  The blocked pass does the
    same measurements with fewer operations (the phase terms are summed once
    per block of 32); the count stays the method's, so that the two kernels
    are measured on one scale."""
    W = (2 * n + 63) // 64
    nr, nd = counters["random"], counters["deterministic"]
    sup = (counters["alg_bytes"] - nr * (24 * W + 80 * n) - nd * 8 * n * W) // (8 * W)
    ops_step = 4 * W * sup
    ops_launch = steps * ops_step / max(1, launches)
    avg_s = sweep_ms * 1e-3 / max(1, launches)
    achieved = ops_launch / avg_s / 1e12 if avg_s > 0 else 0.0
    sweep_bytes = counters["alg_bytes"] - (8 * W * 3 + 80 * n) * nr
    return {
        "kernel": ("k_blk (blocked measurement pass: 32 random measurements per low-rank update, one launch "
                   "per chunk of measurements)" if blocked else
                   "k_meas_xz (register-resident rowsum sweep, one launch per chunk of measurements)"),
        "bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
        "frac": achieved / VALU_PEAK_TOPS,
        "traffic": traffic,
        "launches": launches, "avg_launch_us": avg_s * 1e6,
        "alg_lane_ops_per_launch": ops_launch,
        "support_sum_per_step": int(sup),
        "effective_alg_gbs": steps * sweep_bytes / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else 0.0,
        "note": "32-bit lane operations 4 W sum(2 s + s_x + s_z) per launch over the launch time; peak "
                "157.3 TFLOP/s fp32 / 2 = 78.6e12 lane ops/s (65.8e12 measured for v_xor_b32 by "
                "cliff_calibrate); effective_alg_gbs = the sweep's HBM-streaming bytes over the same time "
                "(the tableau stays on chip, so this exceeds HBM and is not a roofline)",
    }


def make_circuit(name):
    from inputs import plain_large, plain_mid, plain_small
    return {"small": plain_small, "mid": plain_mid, "large": plain_large}[name]()


def golden_outcomes(name):
    path = os.path.join(ROOT, "tests", "golden", "plain_%s.json" % name)
    if not os.path.exists(path):
        return None
    import numpy as np
    rec = json.load(open(path))
    if "outcomes" not in rec:
        return None
    return np.unpackbits(np.frombuffer(bytes.fromhex(rec["outcomes"]), np.uint8),
                         bitorder="little")


def cpu_baseline(c, budget_s: float):
    """Oracle (as it stands, single thread) on a bounded sample of the workload:
    the full gate phase, then as many measurements of the measure-all phase as
    fit the budget; scaled to circuits/s for all shots (the oracle runs shots
    one after another, each from the post-gate tableau)."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    t = oracle.Tableau(c.n).apply_circuit_gates(c)
    t_gates = time.perf_counter() - t0
    k = 0
    t1 = time.perf_counter()
    while k < c.n and (time.perf_counter() - t0) < budget_s:
        t.measure(int(c.qubits[k]), seed=c.seed, circuit=c.circuit_id, shot=0, m=k)
        k += 1
    t_meas = time.perf_counter() - t1
    per_meas = t_meas / max(1, k)
    per_circuit = t_gates + c.shots * per_meas * len(c.qubits)
    return {
        "value": 1.0 / per_circuit, "unit": "circuits/s", "cores": 1, "kind": "oracle",
        "sample": "gate phase in full (%.1fs) + first %d of %d measurements of shot 0 "
                  "(%.3fs each), scaled to %d shot(s) x %d measurements"
                  % (t_gates, k, len(c.qubits), per_meas, c.shots, len(c.qubits)),
        "seconds": time.perf_counter() - t0,
        "host": _host_cpu(),
    }


def bench_plain(P, torch, np, name, steps, warmup, cpu_budget):
    """One of the plain single-circuit workloads (n = 64 or n = 1,024): the
    step of the headline leg (init, encoded layers already in HBM, measure all
    shots, outcomes to the host), circuits/s over `steps` steps, outcomes of
    every shot against the oracle (run live for n = 64, stored for all 128
    shots of n = 1,024), and the oracle's own rate on a bounded sample."""
    c = make_circuit(name)
    ctx = P.Context(0)
    tab = P.DeviceTableau(ctx, c.n, c.shots, init=False)
    ops, offs = P.cliff_encode_layers(c.n, c.h, c.s, c.ctrl, c.tgt)
    dev_ops = torch.from_numpy(ops.view(np.int64)).to("cuda:0")
    torch.cuda.synchronize()

    def step():
        P.cliff_tab_init_zero(tab.handle)
        P.cliff_apply_encoded(tab.handle, dev_ops.data_ptr(), offs)
        return P.cliff_measure(tab.handle, c.qubits, c.seed, c.circuit_id, 0, 0)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out, rnd = step()
    wall = (time.perf_counter() - t0) / steps
    parity = None
    if name == "small":
        import oracle
        parity = all(bool(np.array_equal(out[s], oracle.run_shot(c, s)[0])) for s in range(c.shots))
    else:
        rec = json.load(open(os.path.join(ROOT, "tests", "golden", "plain_mid.json")))
        parity = all(bool(np.array_equal(out[int(s)], np.unpackbits(np.frombuffer(bytes.fromhex(v["outcomes"]),
                                                                                  np.uint8), bitorder="little")[:c.n]))
                     for s, v in rec["shots"].items())
    tab.close()
    ctx.close()
    return {"workload": WORKLOADS[name]["desc"], "circuits_per_s": 1.0 / wall, "us_per_circuit": wall * 1e6,
            "steps": steps, "random_measurements": int(rnd.sum()),
            "parity_all_shots_vs_oracle": parity,
            "cpu_baseline": cpu_baseline(c, cpu_budget) if cpu_budget else None}


def bench_batch(P, torch, np, count=4096, plain_sample=48, reps=5):
    """Batched workload: all circuits in one graph-captured sequence of
    persistent launches vs the plain path (one circuit at a time through the
    HBM kernels) on a sample of the same circuits; outcomes compared bit-exact.
    The plain path is timed twice: on the wall clock with a tableau
    allocation, host encoding and upload per circuit, and kernel-only (op
    streams pre-encoded and resident, tableaux pre-bound, every circuit
    enqueued on one stream and timed with HIP events on it)."""
    from inputs import batch_workload
    from paper_2408_00384_amd.batch import BatchPlan
    t0 = time.perf_counter()
    circs = batch_workload(count)
    gen_s = time.perf_counter() - t0
    stream = torch.cuda.Stream()
    ctx = P.Context(0, stream)
    with torch.cuda.stream(stream):
        plan = BatchPlan(ctx, circs).capture()
        plan.run()
        ctx.sync()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t1 = time.perf_counter()
        ev0.record(stream)
        for _ in range(reps):
            plan.run()
        ev1.record(stream)
        ctx.sync()
        wall = (time.perf_counter() - t1) / reps
        ev_ms = ev0.elapsed_time(ev1) / reps
        outs = plan.outcomes()
    status = plan.status()
    buckets = [{k: b[k] for k in ("edge", "team", "maxn", "max_shots", "count")} for b in plan.buckets]
    lds_bytes = batch_lds_bytes(plan, np)
    head = {
        "workload": "%d circuits, n ~ U{8..256}, depth ~ U{n..4n}, measure all, 4 shots" % count,
        "circuits_per_s": count / (ev_ms * 1e-3),
        "ms_per_batch": ev_ms, "ms_per_batch_wall": wall * 1e3,
        "device_checks": status,
        "buckets": buckets,
    }
    if plain_sample == 0:
        plan.close()
        ctx.close()
        head["lds_alg_bytes_per_batch"] = lds_bytes
        return head
    lds_meas = P.cliff_calibrate(ctx.handle, P.CAL_LDS) / 1e9
    valu_meas = P.cliff_calibrate(ctx.handle, P.CAL_VALU)
    # plain path on an evenly spaced sample
    idx = np.linspace(0, count - 1, plain_sample).astype(int)
    pctx = P.Context(0)
    parity = True
    t2 = time.perf_counter()
    for i in idx:
        c = circs[i]
        tab = P.DeviceTableau(pctx, c.n, c.shots)
        tab.apply_circuit_gates(c)
        o, _ = tab.measure(c.qubits, seed=c.seed, circuit=c.circuit_id)
        parity &= bool(np.array_equal(o, outs[i]))
        tab.close()
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t2) / len(idx)
    # kernel-only plain path: everything resident, one stream, events around it
    kstream = torch.cuda.Stream()
    kctx = P.Context(0, kstream)
    ktabs, kops = [], []
    for i in idx:
        c = circs[i]
        ops, offs = P.cliff_encode_layers(c.n, c.h, c.s, c.ctrl, c.tgt)
        kops.append((torch.from_numpy(ops.view(np.int64)).to("cuda:0"), offs))
        ktabs.append(P.DeviceTableau(kctx, c.n, c.shots, init=False))
    torch.cuda.synchronize()

    def plain_kernels():
        for i, t, (d, offs) in zip(idx, ktabs, kops):
            c = circs[i]
            P.cliff_tab_init_zero(t.handle)
            P.cliff_apply_encoded(t.handle, d.data_ptr(), offs)
            P.cliff_measure_async(t.handle, c.qubits, c.seed, c.circuit_id, 0, 0)

    with torch.cuda.stream(kstream):
        plain_kernels()   # warm-up
        kctx.sync()
        k0, k1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        k0.record(kstream)
        plain_kernels()
        k1.record(kstream)
        kctx.sync()
    plain_kernel_s = k0.elapsed_time(k1) * 1e-3 / len(idx)
    for i, t in zip(idx, ktabs):
        o, _ = P.cliff_tab_read_outcomes(t.handle, len(circs[i].qubits))
        parity &= bool(np.array_equal(o, outs[i]))
        t.close()
    kctx.close()
    pctx.close()
    # the plain path's time depends on n: weight the sample to the whole batch
    ns = np.array([c.n for c in circs])
    plan.close()
    ctx.close()
    return {
        **head,
        "plain_circuits_per_s": 1.0 / plain_s,
        "plain_kernel_circuits_per_s": 1.0 / plain_kernel_s,
        "plain_sample": "%d evenly spaced circuits (mean n %.0f vs %.0f in the batch), one at a time"
                        % (len(idx), ns[idx].mean(), ns.mean()),
        "batched_vs_plain": (count / (ev_ms * 1e-3)) * plain_s,
        "batched_vs_plain_kernel": (count / (ev_ms * 1e-3)) * plain_kernel_s,
        "plain_timing": "batched_vs_plain: plain path on the wall clock, a tableau allocated, gates encoded on "
                        "the host and uploaded per circuit; batched_vs_plain_kernel: op streams pre-encoded in "
                        "HBM, tableaux pre-bound, all circuits enqueued on one stream, HIP events around them",
        "bit_exact_vs_plain": parity,
        "lds": {"alg_bytes_per_batch": lds_bytes, "achieved_gbs": lds_bytes / (ev_ms * 1e-3) / 1e9,
                "peak_gbs": LDS_PEAK_GBS, "frac": lds_bytes / (ev_ms * 1e-3) / 1e9 / LDS_PEAK_GBS,
                "measured_peak_gbs": lds_meas,
                "frac_of_measured": lds_bytes / (ev_ms * 1e-3) / 1e9 / lds_meas,
                "note": "tableaux live in LDS; algorithmic LDS bytes of the gate updates and "
                        "measurement sweeps over the whole batch time; measured peak: cliff_calibrate "
                        "(conflict-free 16-byte reads on every CU)"},
        "valu_measured_lane_ops_per_s": valu_meas,
        "cpu_baseline": batch_cpu_baseline(circs, np),
        "generate_s": gen_s,
    }


def _oracle_circuit(c):
    import oracle
    t = oracle.Tableau(c.n).apply_circuit_gates(c)
    for s in range(c.shots):
        t.clone().measure_list(c.qubits, seed=c.seed, circuit=c.circuit_id, shot=s)


def batch_cpu_baseline(circs, np, sample: int = 512):
    """The oracle on an evenly spaced sample of the batch, every shot of every
    circuit (gates once, each shot from the post-gate tableau), one circuit per
    thread on the host's cores (the oracle's C calls release the GIL)."""
    import concurrent.futures as cf
    import oracle
    oracle.build(force=False)
    idx = np.linspace(0, len(circs) - 1, min(sample, len(circs))).astype(int)
    workers = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda i: _oracle_circuit(circs[i]), idx))
    wall = time.perf_counter() - t0
    ns = np.array([c.n for c in circs])
    return {"value": len(idx) / wall, "unit": "circuits/s", "cores": workers, "kind": "oracle",
            "sample": "%d evenly spaced circuits of the batch (mean n %.0f vs %.0f), all shots, one circuit "
                      "per thread on %d threads" % (len(idx), ns[idx].mean(), ns.mean(), workers),
            "seconds": wall, "host": _host_cpu()}


def _oracle_request_seconds(c, gate_s, meas_s):
    """One thread's oracle time for one serving request, from a bounded run:
    gate layers in order until gate_s is spent, the rest scaled by layer count
    (a layer costs the same in any state: every gate sweeps all 2n rows, one
    byte per bit); then measurements of shot 0 until meas_s is spent, scaled
    to all n measurements of every shot (the oracle runs shots one after
    another from the post-gate tableau).  Returns (seconds, layers, measured)."""
    import oracle
    t = oracle.Tableau(c.n)
    depth = c.h.shape[0]
    t0 = time.perf_counter()
    done = 0
    while done < depth and (done == 0 or time.perf_counter() - t0 < gate_s):
        l1 = min(depth, done + 4)
        t.apply_layers(c.h[done:l1], c.s[done:l1], c.ctrl[done:l1], c.tgt[done:l1])
        done = l1
    gates = (time.perf_counter() - t0) * depth / max(1, done)
    t1 = time.perf_counter()
    k = 0
    while k < len(c.qubits) and (k == 0 or time.perf_counter() - t1 < meas_s):
        t.measure(int(c.qubits[k]), seed=c.seed, circuit=c.circuit_id, shot=0, m=k)
        k += 1
    meas = (time.perf_counter() - t1) / max(1, k) * len(c.qubits) * c.shots
    return gates + meas, done, k


def serving_cpu_baseline(circs, np, gate_s: float = 1.0, meas_s: float = 1.0):
    """The oracle's rate on the serving requests with one request per thread
    on the host's cores: every request's single-thread time from a bounded run
    (`_oracle_request_seconds`), summed and spread evenly over the threads."""
    import concurrent.futures as cf
    import oracle
    oracle.build(force=False)
    workers = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(workers) as ex:
        res = list(ex.map(lambda c: _oracle_request_seconds(c, gate_s, meas_s), circs))
    wall = time.perf_counter() - t0
    secs = np.array([r[0] for r in res])
    full = sum(1 for c, r in zip(circs, res) if r[1] == c.h.shape[0] and r[2] == len(c.qubits))
    return {"value": float(len(circs) / (secs.sum() / workers)), "unit": "circuits/s", "cores": workers, "kind": "oracle",
            "sample": "all %d requests, one per thread on %d threads; per request the gate layers of the first "
                      "%.1f s and the shot-0 measurements of the next %.1f s, scaled to the full depth and to n "
                      "measurements x shots (gates and shot 0 complete for %d requests); rate = requests / (summed seconds / threads)"
                      % (len(circs), workers, gate_s, meas_s, full),
            "oracle_seconds_total": float(secs.sum()), "seconds": wall, "host": _host_cpu()}


def batch_lds_bytes(plan, np):
    """Algorithmic LDS bytes of a batch: per row word (64 rows, 8 bytes per
    plane) a two-qubit op reads and writes x and z of two columns (64 B), a
    single-qubit op of one (32 B); every measurement sweeps all n columns,
    reading the pivot row's bits and x, z and writing x, z (48 B per column
    and row word; measurements counted as random, as nearly all are in these
    dense states)."""
    n = plan.descs["n"].astype(np.int64)
    W = (2 * n + 63) // 64
    gates = (64 * plan.pair_count + 32 * (plan.op_count - plan.pair_count)) * W
    meas = 48 * n * n * W
    return int(gates.sum() + meas.sum())


def _gen_clifford(args):
    from inputs import random_clifford
    n, seed, i = args
    c = random_clifford(n, [seed, n, i], circuit_id=i)
    return c.ops, c.a, c.b


def _tab_digest(x, z, r):
    h = hashlib.sha256()
    for a in (x, z, r):
        h.update(a.tobytes())
    return h.hexdigest()


FIG2A_NS = tuple(range(100, 1001, 100))


def gen_cliffords(ns, count=100, seed=5):
    """Circuit i of size n: generator seed [seed, n, i].  Drawn in worker
    processes forked before this process touches the GPU (so no child
    inherits GPU state, and the pool leaves no helper process behind)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    workers = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
        lists = list(ex.map(_gen_clifford, [(n, seed, i) for n in ns for i in range(count)]))
    out = {n: lists[k * count:(k + 1) * count] for k, n in enumerate(ns)}
    return out, time.perf_counter() - t0


def bench_clifford(P, torch, np, n, lists, seed=5, reps=3, oracle_circuits=1):
    """The paper's Fig. 2a workload at one n: uniformly random Clifford
    circuits on n qubits, gates only, from |0...0>.  Op streams resident in
    HBM; one many-tableau launch for all circuits vs one launch per circuit
    (plain); tableaux compared bit for bit between the two, and against the
    oracle's stored digests where they exist; the oracle timed on
    `oracle_circuits` circuits."""
    import concurrent.futures as cf
    count = len(lists)
    workers = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(workers) as ex:   # the encoder runs without the GIL
        enc = list(ex.map(lambda l: P.cliff_encode_gates(n, *l), lists))
    enc_s = time.perf_counter() - t0
    gates = sum(len(l[0]) for l in lists)
    layers = [len(o) - 1 for _, o in enc]
    stream = torch.cuda.Stream()
    ctx = P.Context(0, stream)
    dev = [torch.from_numpy(w.view(np.int64)).to("cuda:0") for w, _ in enc]
    offs = [o for _, o in enc]
    ptrs = [d.data_ptr() for d in dev]
    torch.cuda.synchronize()
    tabs = [P.DeviceTableau(ctx, n, 1) for _ in range(count)]
    handles = [t.handle for t in tabs]

    def batched():
        for t in tabs:
            t.init_zero()
        P.cliff_apply_encoded_many(handles, ptrs, offs)

    def plain():
        for t, p, o in zip(tabs, ptrs, offs):
            t.init_zero()
            P.cliff_apply_encoded(t.handle, p, o)

    res = {}
    digests = {}
    with torch.cuda.stream(stream):
        for name, fn in (("batched", batched), ("plain", plain)):
            fn()   # warm-up
            ctx.sync()
            P.cliff_ctx_profile(ctx.handle, True)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t1 = time.perf_counter()
            ev0.record(stream)
            for _ in range(reps):
                fn()
            ev1.record(stream)
            ctx.sync()
            wall = (time.perf_counter() - t1) / reps
            gate_ms, launches = P.cliff_ctx_profile_read(ctx.handle, "gate")
            P.cliff_ctx_profile(ctx.handle, False)
            ms = ev0.elapsed_time(ev1) / reps
            res[name] = {"circuits_per_s": count / (ms * 1e-3), "ms": ms, "ms_wall": wall * 1e3,
                         "gate_kernel_ms": gate_ms / reps, "gate_launches": launches // reps}
            digests[name] = []
            for t in tabs:
                x, z, r = t.export()
                digests[name].append(_tab_digest(x, z, r[0]))
    for t in tabs:
        t.close()
    ctx.close()
    golden = os.path.join(ROOT, "tests", "golden", "clifford_n%d.json" % n)
    vs_oracle = None
    if os.path.exists(golden) and seed == 5:
        rec = json.load(open(golden))["circuits"]
        vs_oracle = all(digests["batched"][int(i)] == v["tableau_sha256"] for i, v in rec.items()
                        if int(i) < count)
    cpu = None
    if oracle_circuits:
        import oracle
        t2 = time.perf_counter()
        for i in range(oracle_circuits):
            oracle.Tableau(n).apply_gates(*lists[i])
        cpu_s = (time.perf_counter() - t2) / oracle_circuits
        cpu = {"circuits_per_s": 1.0 / cpu_s, "cores": 1, "kind": "oracle",
               "sample": "%d of the %d circuits, gates only" % (oracle_circuits, count)}
    b = res["batched"]
    return {
        "n": n, "circuits": count,
        "circuits_per_s": b["circuits_per_s"],
        "gates_per_circuit": gates / count,
        "layers_per_circuit": float(np.mean(layers)),
        "row_gate_updates_per_s": gates * 2 * n / (b["ms"] * 1e-3),
        "batched": b,
        "plain": res["plain"],
        "batched_vs_plain": b["circuits_per_s"] / res["plain"]["circuits_per_s"],
        "bit_exact_batched_vs_plain": digests["batched"] == digests["plain"],
        "bit_exact_vs_oracle_stored": vs_oracle,
        "cpu_baseline": cpu,
        "encode_s": enc_s,
    }


def bench_fig2a(P, torch, np, lists_by_n, gen_s):
    """Fig. 2a's curve: 100 uniformly random Cliffords per n, n = 100..1000."""
    rows = []
    for n in sorted(lists_by_n):
        print("#   n = %d" % n, file=sys.stderr, flush=True)
        rows.append(bench_clifford(P, torch, np, n, lists_by_n[n]))
    return {"workload": "100 uniformly random Clifford circuits (Bravyi-Maslov canonical form) per n, gates "
                        "only, from |0...0>; circuit i of size n from generator seed [5, n, i]",
            "generate_s": gen_s, "per_n": rows}


def bench_xlarge(P, torch, np, k=256, reps=2):
    """The HBM-bound path beyond the Infinity Cache: n = 25,000 (a 313 MB
    tableau; the register-resident path holds at most n = 10,240), gates, then
    qubits 0..k-1 measured, one per-measurement kernel each.  Reports the
    sweep kernels' algorithmic HBM bandwidth (device counters over HIP-event
    kernel time); the first 32 outcomes are compared with the oracle's."""
    from inputs import plain_xlarge
    c = plain_xlarge()
    ctx = P.Context(0)
    tab = P.DeviceTableau(ctx, c.n, 1, init=False)
    ops, offs = P.cliff_encode_layers(c.n, c.h, c.s, c.ctrl, c.tgt)
    dev_ops = torch.from_numpy(ops.view(np.int64)).to("cuda:0")
    torch.cuda.synchronize()
    q = np.arange(k, dtype=np.uint32)
    n, W = c.n, (2 * c.n + 63) // 64
    best = None
    for rep in range(reps + 1):
        P.cliff_tab_init_zero(tab.handle)
        P.cliff_apply_encoded(tab.handle, dev_ops.data_ptr(), offs)
        ctx.sync()
        P.cliff_ctx_profile(ctx.handle, True)
        t0 = time.perf_counter()
        out, rnd = P.cliff_measure(tab.handle, q, c.seed, c.circuit_id, 0, 0)
        wall = time.perf_counter() - t0
        prof = {kk: P.cliff_ctx_profile_read(ctx.handle, kk) for kk in P.PROF_KINDS}
        P.cliff_ctx_profile(ctx.handle, False)
        if rep and (best is None or wall < best[0]):
            best = (wall, prof, P.cliff_tab_counters(tab.handle), out, rnd)
    wall, prof, counters, out, rnd = best
    nr = counters["random"]
    sweep_bytes = counters["alg_bytes"] - (8 * W * 3 + 80 * n) * nr
    sweep_ms, launches = prof["sweep"]
    gbs = sweep_bytes / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else 0.0
    parity = None
    gold = os.path.join(ROOT, "tests", "golden", "plain_xlarge_prefix.json")
    if os.path.exists(gold):
        rec = json.load(open(gold))
        kk = rec["k"]
        def bits(h):
            return np.unpackbits(np.frombuffer(bytes.fromhex(h), np.uint8), bitorder="little")[:kk]
        parity = bool(np.array_equal(out[0][:kk], bits(rec["outcomes"])) and
                      np.array_equal(rnd[:kk], bits(rec["random"])))
    tab.close()
    ctx.close()
    return {
        "workload": "n = 25,000, 20 layers (generator seed 6), qubits 0..%d measured, 1 shot" % (k - 1),
        "tableau_bytes": 2 * n * W * 8,
        "measurements": k, "random": int(nr), "ms_measure": wall * 1e3,
        "us_per_measurement": wall * 1e6 / k,
        "sweep": {"kernel": "k_step (one launch per measurement)", "launches": launches,
                  "ms": sweep_ms, "alg_bytes": sweep_bytes, "alg_gbs": gbs, "frac_of_8000": gbs / HBM_PEAK_GBS},
        "parity_first_32_vs_stored_oracle": parity,
    }


def bench_serving(P, np, count=1000, sat_count=200, cpu_count=96, seed=4, budget=64 << 30, lanes=8,
                  cpu=True):
    """Serving workload: n log-uniform in [16, 4096], depth 2n, shots in
    [1, 1024], admission against a 64 GB budget.  A closed-loop pass over the
    first `sat_count` requests (every one admitted at once) gives the
    saturated throughput; then all `count` requests arrive as a Poisson
    stream at 70% of it, for the latencies; the requests served in both
    passes must give the same outcomes.  The oracle is timed on the first
    `cpu_count` requests."""
    from inputs import serving_params, serving_request
    from paper_2408_00384_amd.serving import Server, summarize
    arrivals, ns, shots = serving_params(count, 1.0, seed=seed)
    circs = [serving_request(i, arrivals, ns, shots, seed=seed).circuit for i in range(count)]
    srv = Server(budget_bytes=budget, lanes=lanes)
    t0 = time.perf_counter()
    sat = srv.run(circs[:sat_count], np.zeros(sat_count), realtime=False)
    sat_s = time.perf_counter() - t0
    sat_rate = sat_count / sat_s
    rate = 0.7 * sat_rate
    print("#   saturated %.1f requests/s; Poisson at %.1f/s over %d requests" % (sat_rate, rate, count),
          file=sys.stderr, flush=True)
    arrivals = np.asarray(arrivals) / rate   # the same unit-rate draws, scaled to `rate`
    mix = srv.run(circs, arrivals, realtime=True)
    same = all(np.array_equal(sat[i].outcomes, mix[i].outcomes) for i in range(sat_count)
               if sat[i].error is None)
    st = summarize(mix)
    peak = srv.alloc.peak
    srv.close()
    return {
        "workload": "%d requests, n log-uniform [16, 4096], depth 2n, shots U{1..1024}, "
                    "64 GB admission budget, %d HBM lanes + 1 batch lane" % (count, lanes),
        "saturated_circuits_per_s": sat_rate,
        "saturated_sample": "closed loop over the first %d requests" % sat_count,
        "poisson_rate_hz": rate,
        "latency_samples": st["completed"],
        "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
        "circuits_per_s": st["circuits_per_s"],
        "paths": st["paths"], "rejected": st["rejected"],
        "arena_peak_bytes": peak,
        "outcomes_same_as_closed_loop": same,
        "max_n": int(max(ns)), "total_shots": int(sum(shots)),
        "cpu_baseline": serving_cpu_baseline(circs[:cpu_count], np) if cpu else None,
    }


def _host_cpu():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip() + ", %d logical CPUs" % os.cpu_count()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-circuits leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-clifford", action="store_true",
                    help="skip the uniform-random-Clifford (gates only) sweep over n")
    ap.add_argument("--no-plain-legs", action="store_true",
                    help="skip the n = 64 and n = 1,024 workloads")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving leg (for a kernel trace of it); prints its JSON")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched leg, without its plain-path comparisons and oracle "
                         "baseline (for kernel traces and counters of the batch kernel); prints its JSON")
    ap.add_argument("--no-xlarge", action="store_true",
                    help="skip the n = 25,000 HBM-bound measurement leg")
    ap.add_argument("--no-profile", action="store_true",
                    help="no per-kernel HIP events (for hardware-counter runs); no roofline")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device-to-device 4 times (known bytes, to scale HBM counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        nbytes = 1 << 30
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record()
        for i in range(4):
            dst.copy_(src)
            ev[i + 1].record()
        torch.cuda.synchronize()
        ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(4)]
        # read + write bytes over the fastest copy's time
        print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": 4,
                          "copy_ms": ms, "copy_gbs_read_plus_write": 2 * nbytes / (min(ms) * 1e-3) / 1e9}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: measures one GPU only (the tableau hot path is "
              "single-GPU); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # circuits of the Fig. 2a sweep, drawn before anything touches the GPU
    fig2a_lists, fig2a_gen_s = None, 0.0
    if not (args.no_clifford or args.serving_only or args.batch_only):
        print("# drawing uniformly random Cliffords for n = %s ..." % (FIG2A_NS,), file=sys.stderr, flush=True)
        fig2a_lists, fig2a_gen_s = gen_cliffords(FIG2A_NS)

    import numpy as np
    import torch
    import paper_2408_00384_amd as P

    if args.serving_only:
        print(json.dumps({"serving": bench_serving(P, np, cpu=False)}), flush=True)
        torch.cuda.synchronize()
        return
    if args.batch_only:
        print(json.dumps({"batched": bench_batch(P, torch, np, plain_sample=0)}), flush=True)
        torch.cuda.synchronize()
        return

    wl = WORKLOADS[args.workload]
    steps = args.steps if args.steps is not None else wl["steps"]
    warmup = args.warmup if args.warmup is not None else wl["warmup"]
    c = make_circuit(args.workload)
    print("# workload %s: %s" % (args.workload, wl["desc"]), file=sys.stderr, flush=True)

    ctx = P.Context(0)
    tab = P.DeviceTableau(ctx, c.n, c.shots, init=False)
    ops, offs = P.cliff_encode_layers(c.n, c.h, c.s, c.ctrl, c.tgt)
    dev_ops = torch.from_numpy(ops.view(np.int64)).to("cuda:0")
    torch.cuda.synchronize()
    qubits = c.qubits

    def step():
        P.cliff_tab_init_zero(tab.handle)
        P.cliff_apply_encoded(tab.handle, dev_ops.data_ptr(), offs)
        return P.cliff_measure(tab.handle, qubits, c.seed, c.circuit_id, 0, 0)

    for i in range(warmup):
        step()
        print("# warmup %d done" % (i + 1), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    # per-kernel HIP events on the library's stream for every launch of the
    # timed steps (a few microseconds per launch of overhead)
    if not args.no_profile:
        P.cliff_ctx_profile(ctx.handle, True)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    out = rnd = None
    for i in range(steps):
        out, rnd = step()
        print("# step %d done" % (i + 1), file=sys.stderr, flush=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = ev0.elapsed_time(ev1)
    ms_per_step = wall * 1e3 / steps

    # parity against stored oracle outcomes (if present) -- bit exact
    gold = golden_outcomes(args.workload)
    parity = None
    if gold is not None and c.shots == 1:
        parity = bool(np.array_equal(out[0], gold[: c.n]))

    prof = {k: P.cliff_ctx_profile_read(ctx.handle, k) for k in P.PROF_KINDS}
    if not args.no_profile:
        P.cliff_ctx_profile(ctx.handle, False)
    # device counters cover the last step (init clears them); steps are identical
    counters = P.cliff_tab_counters(tab.handle)
    n, W = c.n, (2 * c.n + 63) // 64
    nr, nd = counters["random"], counters["deterministic"]
    alg_step = counters["alg_bytes"]
    # the sweep kernel's share: x/z words of the pivot-touching columns
    # (random) and the stabilizer halves (deterministic); the update mask,
    # counter planes and row rewrites belong to the finalize kernels
    sweep_step = alg_step - (8 * W * 3 + 80 * n) * nr
    sweep_ms, sweep_launches = prof["sweep"]
    blk_ms, blk_launches = prof["blocked"]
    persistent = sweep_launches < steps * len(qubits)
    meas_ms = sum(prof[k][0] for k in ("select", "sweep", "final", "blocked"))
    if blk_launches and blk_ms > sweep_ms:
        roofline = alu_roofline(counters, n, steps, blk_ms, blk_launches,
                                traffic_for("k_blk") if args.workload == "large" else None, blocked=True)
    elif persistent:
        roofline = alu_roofline(counters, n, steps, sweep_ms, sweep_launches,
                                traffic_for("k_meas_xz") if args.workload == "large" else None)
    else:
        achieved = steps * sweep_step / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else 0.0
        roofline = {"kernel": "k_step (rowsum sweep, one launch per measurement)",
                    "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "launches": sweep_launches, "avg_launch_us": 1e3 * sweep_ms / max(1, sweep_launches),
                    "alg_bytes_per_launch": steps * sweep_step / max(1, sweep_launches)}
    tab.close()
    ctx.close()
    print("# kernels over %d steps: " % steps
          + ", ".join("%s %.2f ms/%d" % (k, v[0], v[1]) for k, v in prof.items()),
          file=sys.stderr, flush=True)

    result = {
        "metric": "Clifford circuits/s batched vs plain (bit-exact) + tableau sweep HBM GB/s",
        "value": 1e3 / ms_per_step,
        "unit": "circuits/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_hip_events": ev_ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "n": c.n, "layers": c.depth, "shots": c.shots,
                   "measurements": int(len(c.qubits)), "random_measurements": int(rnd.sum()),
                   "generator_seed": {"small": 0, "mid": 1, "large": 2}[args.workload]},
        "parity_vs_stored_oracle": parity,
        "roofline": roofline,
        "measure_phase": {
            "alg_bytes_per_step": alg_step,
            "ms_per_step": meas_ms / steps,
            "alg_gbs": alg_step / (meas_ms / steps * 1e-3) / 1e9 if meas_ms > 0 else 0.0,
        },
        "kernel_ms_per_step": {k: round(v[0] / steps, 3) for k, v in prof.items()},
        "anomalies": counters["anomalies"],
    }
    if args.no_profile:
        result["roofline"] = None
        result.pop("measure_phase")
    if not args.no_plain_legs:
        budget = 0.0 if args.no_cpu_baseline else 10.0
        for name in ("small", "mid"):
            if name == args.workload:
                continue
            print("# plain %s ..." % name, file=sys.stderr, flush=True)
            result["plain_" + name] = bench_plain(P, torch, np, name, WORKLOADS[name]["steps"],
                                                  WORKLOADS[name]["warmup"], budget)
    if not args.no_batch:
        print("# batched circuits ...", file=sys.stderr, flush=True)
        result["batched"] = bench_batch(P, torch, np)
    if not args.no_serving:
        print("# serving ...", file=sys.stderr, flush=True)
        result["serving"] = bench_serving(P, np, cpu=not args.no_cpu_baseline)
    if not args.no_clifford:
        print("# uniform random Cliffords, gates only, n = 100..1000 ...", file=sys.stderr, flush=True)
        result["fig2a"] = bench_fig2a(P, torch, np, fig2a_lists, fig2a_gen_s)
        result["random_clifford"] = result["fig2a"]["per_n"][-1]   # n = 1000
    if not args.no_xlarge:
        print("# n = 25,000, per-measurement kernels ...", file=sys.stderr, flush=True)
        result["xlarge_hbm"] = bench_xlarge(P, torch, np)
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(c, args.cpu_budget)
    torch.cuda.synchronize()   # every context and tableau above is closed; nothing is left in flight
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

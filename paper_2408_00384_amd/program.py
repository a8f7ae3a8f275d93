"""Runner for circuits with mid-circuit measurement, reset and classically
conditioned Paulis (the step format of ``inputs.programs``).

All shots run together on one tableau with one sign column per shot: a
measurement's outcomes go to a device record (one byte per shot and
measurement), a reset is a measurement plus an X in the shots that read 1,
and a conditioned Pauli flips signs in the shots whose recorded bit is 1.
None of these changes X/Z differently per shot, so the shots keep sharing one
X/Z sweep.  A gate list conditioned on a recorded bit ("cgates") does change
X/Z per shot: a program with one runs every shot on a tableau of its own
(gate lists for all shots in one many-tableau launch, the conditioned ones
for the shots whose bit is 1), with each shot's own index as the random-bit
shot index, so both modes give the same outcomes shot by shot.  Every step
runs in the library's kernels; this module only walks the step list and owns
the record's device memory.
"""
from __future__ import annotations

import collections

import numpy as np
import torch

from . import _binding as B
from .device import Context, DeviceTableau


def run_program(ctx: Context, prog, tab: "DeviceTableau | None" = None):
    """Run ``prog`` on all its shots from |0...0> (or on ``tab`` as it
    stands).  Returns (record uint8[shots, M], random flags uint8[M], tab);
    for a program with conditioned gate lists (record, random flags
    uint8[shots, M], list of per-shot tableaux)."""
    if any(st[0] == "cgates" for st in prog.steps):
        if tab is not None:
            raise ValueError("a program with conditioned gate lists runs on per-shot tableaux")
        return _run_per_shot(ctx, prog)
    if tab is None:
        tab = DeviceTableau(ctx, prog.n, prog.shots)
    S, M = tab.shots, prog.measurements
    dev = "cuda:%d" % ctx.device
    with torch.cuda.stream(ctx.stream):
        rec = torch.zeros((S, max(1, M)), dtype=torch.uint8, device=dev)
        rnd = torch.zeros(max(1, M), dtype=torch.uint8, device=dev)
    ld = rec.shape[1]
    col = 0
    for st in prog.steps:
        kind = st[0]
        if kind == "gates":
            tab.apply_gates(st[1], st[2], st[3])
        elif kind in ("measure", "reset"):
            fn = B.cliff_measure_record if kind == "measure" else B.cliff_reset_record
            fn(tab.handle, st[1], rec.data_ptr(), ld, col, rnd.data_ptr(), seed=prog.seed,
               circuit=prog.circuit_id, m0=col)
            col += len(st[1])
        elif kind == "cond":
            B.cliff_apply_cond_paulis(tab.handle, st[1], st[2], st[3], rec.data_ptr(), ld)
        else:
            raise ValueError("unknown program step %r" % (kind,))
    ctx.sync()
    tab.anomalies()     # raises if a register-resident measurement gave up
    return rec[:, :M].cpu().numpy(), rnd[:M].cpu().numpy(), tab


def _run_per_shot(ctx: Context, prog):
    S, M, n = prog.shots, prog.measurements, prog.n
    tabs = [DeviceTableau(ctx, n, 1) for _ in range(S)]
    handles = [t.handle for t in tabs]
    dev = "cuda:%d" % ctx.device
    with torch.cuda.stream(ctx.stream):
        rec = torch.zeros((S, max(1, M)), dtype=torch.uint8, device=dev)
        rnd = torch.zeros((S, max(1, M)), dtype=torch.uint8, device=dev)
    ld = rec.shape[1]
    many = n <= 20352          # the many-tableau launch holds 2 n 4 bytes of LDS at 32 rows

    def gates(sel, ops, a, b):
        if not sel:
            return
        if many:
            B.cliff_apply_gates_many([handles[s] for s in sel], [(ops, a, b)] * len(sel), 0)
        else:
            for s in sel:
                tabs[s].apply_gates(ops, a, b)

    col = 0
    for st in prog.steps:
        kind = st[0]
        if kind == "gates":
            gates(list(range(S)), st[1], st[2], st[3])
        elif kind in ("measure", "reset"):
            fn = B.cliff_measure_record if kind == "measure" else B.cliff_reset_record
            for s in range(S):   # shot s: row s of the record, random-bit shot index s
                fn(handles[s], st[1], rec.data_ptr() + s * ld, ld, col, rnd.data_ptr() + s * ld,
                   seed=prog.seed, circuit=prog.circuit_id, shot0=s, m0=col)
            col += len(st[1])
        elif kind == "cond":
            for s in range(S):
                B.cliff_apply_cond_paulis(handles[s], st[1], st[2], st[3], rec.data_ptr() + s * ld, ld)
        elif kind == "cgates":
            ctx.sync()
            bits = rec[:, int(st[1])].cpu().numpy()
            gates([s for s in range(S) if bits[s]], st[2], st[3], st[4])
        else:
            raise ValueError("unknown program step %r" % (kind,))
    ctx.sync()
    for t in tabs:
        t.anomalies()   # raises if a register-resident measurement gave up
    return rec[:, :M].cpu().numpy(), rnd[:, :M].cpu().numpy(), tabs


def outcome_counts(record: np.ndarray) -> "collections.Counter[str]":
    """Frequencies of the shots' outcome strings ('0'/'1' per recorded
    measurement, in record order)."""
    rows = np.ascontiguousarray(record, np.uint8)
    keys, counts = np.unique(rows, axis=0, return_counts=True)
    return collections.Counter({"".join(map(str, k)): int(c) for k, c in zip(keys, counts)})

"""Runner for circuits with mid-circuit measurement, reset and classically
conditioned Paulis (the step format of ``inputs.programs``).

All shots run together on one tableau with one sign column per shot: a
measurement's outcomes go to a device record (one byte per shot and
measurement), a reset is a measurement plus an X in the shots that read 1,
and a conditioned Pauli flips signs in the shots whose recorded bit is 1.
None of these changes X/Z differently per shot, so the shots keep sharing one
X/Z sweep.  Every step runs in the library's kernels; this module only walks
the step list and owns the record's device memory.
"""
from __future__ import annotations

import collections

import numpy as np
import torch

from . import _binding as B
from .device import Context, DeviceTableau


def run_program(ctx: Context, prog, tab: "DeviceTableau | None" = None):
    """Run ``prog`` on all its shots from |0...0> (or on ``tab`` as it
    stands).  Returns (record uint8[shots, M], random flags uint8[M], tab)."""
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
    return rec[:, :M].cpu().numpy(), rnd[:M].cpu().numpy(), tab


def outcome_counts(record: np.ndarray) -> "collections.Counter[str]":
    """Frequencies of the shots' outcome strings ('0'/'1' per recorded
    measurement, in record order)."""
    rows = np.ascontiguousarray(record, np.uint8)
    keys, counts = np.unique(rows, axis=0, return_counts=True)
    return collections.Counter({"".join(map(str, k)): int(c) for k, c in zip(keys, counts)})

"""Seeded circuits with mid-circuit measurement, reset and classically
conditioned Paulis (no tableau arithmetic here: only the instruction lists).

A program on n qubits is a list of steps, run in order on every shot:

  ("gates", ops, a, b)        gate list (op codes of ``inputs.circuits``)
  ("measure", qubits)         Z-measure each qubit in order
  ("reset", qubits)           reset each qubit to |0> (Z-measure, X if 1)
  ("cond", qubits, paulis, cols)
                              apply Pauli paulis[i] (1 X, 2 Y, 3 Z) to
                              qubits[i] in the shots whose recorded outcome
                              in column cols[i] is 1
  ("cgates", col, ops, a, b)  apply the gate list in the shots whose recorded
                              outcome in column col is 1 (any Clifford gates:
                              the shots' X/Z bits then differ)

Every measurement (from "measure" or "reset") takes the next column of the
shot's outcome record; its random-bit index m is that column.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .circuits import PHILOX_SEED, random_gate_list


@dataclasses.dataclass
class Program:
    n: int
    steps: list
    shots: int
    circuit_id: int = 0
    seed: int = PHILOX_SEED

    @property
    def measurements(self) -> int:
        return sum(len(st[1]) for st in self.steps if st[0] in ("measure", "reset"))


def random_program(n: int, blocks: int, shots: int, gen_seed, circuit_id: int = 0,
                   conditioned_gates: bool = False) -> Program:
    """``blocks`` rounds of: a full-gate-set gate list, then a measurement, a
    reset or a set of conditioned Paulis on a few random qubits (conditions on
    columns already recorded), or with ``conditioned_gates`` also a short
    gate list conditioned on a recorded column.  Qubits within one measure or
    reset step may repeat."""
    rng = np.random.Generator(np.random.PCG64(gen_seed))
    steps = []
    cols = 0
    for _ in range(blocks):
        ops, a, b = random_gate_list(rng, n, int(rng.integers(1, 4 * n + 8)), full=True)
        steps.append(("gates", ops, a, b))
        if conditioned_gates and cols and rng.random() < 0.4:
            col = int(rng.integers(0, cols))
            cops, ca, cb = random_gate_list(rng, n, int(rng.integers(1, n + 4)), full=True)
            steps.append(("cgates", col, cops, ca, cb))
            continue
        kind = int(rng.integers(0, 3)) if cols else int(rng.integers(0, 2))
        k = int(rng.integers(1, min(n, 6) + 1))
        q = rng.integers(0, n, size=k).astype(np.uint32)
        if kind == 0:
            steps.append(("measure", q))
            cols += k
        elif kind == 1:
            steps.append(("reset", q))
            cols += k
        else:
            paulis = rng.integers(1, 4, size=k).astype(np.uint8)
            c = rng.integers(0, cols, size=k).astype(np.uint32)
            steps.append(("cond", q, paulis, c))
    return Program(n=n, steps=steps, shots=shots, circuit_id=circuit_id)

"""Seeded synthetic Clifford-circuit workloads.

This module only draws random numbers and arranges them into plain arrays. It
holds none of the stabilizer-tableau arithmetic, so both the CPU oracle and the
GPU path can consume the very same circuits without sharing any simulation code.

Circuit structure (one "layer"): every qubit independently receives H with
probability 1/2, then S with probability 1/2; then CNOTs act on a uniformly
random perfect matching of the qubits, each pair with a random orientation.
For odd n the last qubit of the random permutation idles in the CNOT stage.

The paper benchmarks uniformly random Cliffords (Sec. 2, Fig. 2a caption),
whose sampled circuits are not published; these layered circuits stand in for
them with the sizes of the five workloads below.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Philox key used for the random measurement outcomes of every workload.
PHILOX_SEED = 0x240800384


@dataclasses.dataclass
class Circuit:
    """A layered H/S/CNOT circuit followed by Z-measurement of ``qubits``.

    Arrays (all C-contiguous):
      h, s      uint8  [depth, n]      1 = apply the gate to that qubit
      ctrl, tgt uint32 [depth, n // 2] CNOT control/target per pair
    Layer order: per qubit H then S, then all CNOTs of the layer.
    """

    n: int
    h: np.ndarray
    s: np.ndarray
    ctrl: np.ndarray
    tgt: np.ndarray
    qubits: np.ndarray
    shots: int
    circuit_id: int = 0
    seed: int = PHILOX_SEED

    @property
    def depth(self) -> int:
        return int(self.h.shape[0])

    def gate_count(self) -> int:
        return int(self.h.sum()) + int(self.s.sum()) + int(self.ctrl.size)


def random_layers(rng: np.random.Generator, n: int, depth: int):
    """Draw ``depth`` layers for ``n`` qubits from ``rng``.

    Draw order: all H coins, all S coins, the per-layer permutations, then
    the orientation coins.
    """
    h = rng.integers(0, 2, size=(depth, n), dtype=np.uint8)
    s = rng.integers(0, 2, size=(depth, n), dtype=np.uint8)
    base = np.broadcast_to(np.arange(n, dtype=np.uint32), (depth, n))
    perm = rng.permuted(base, axis=1)
    orient = rng.integers(0, 2, size=(depth, n // 2), dtype=np.uint8)
    first = perm[:, 0 : 2 * (n // 2) : 2]
    second = perm[:, 1 : 2 * (n // 2) : 2]
    ctrl = np.where(orient == 0, first, second).astype(np.uint32)
    tgt = np.where(orient == 0, second, first).astype(np.uint32)
    return (np.ascontiguousarray(h), np.ascontiguousarray(s),
            np.ascontiguousarray(ctrl), np.ascontiguousarray(tgt))


def layered_circuit(n: int, depth: int, shots: int, gen_seed, circuit_id: int = 0,
                    seed: int = PHILOX_SEED) -> Circuit:
    """Random layered circuit measuring every qubit in ascending order."""
    rng = np.random.Generator(np.random.PCG64(gen_seed))
    h, s, ctrl, tgt = random_layers(rng, n, depth)
    return Circuit(n=n, h=h, s=s, ctrl=ctrl, tgt=tgt,
                   qubits=np.arange(n, dtype=np.uint32), shots=shots,
                   circuit_id=circuit_id, seed=seed)


# --- the five workloads -------------------------------------------------------

def plain_small() -> Circuit:
    """n = 64, 64 layers, measure all 64 qubits, 16 shots (generator seed 0)."""
    return layered_circuit(64, 64, 16, gen_seed=0)


def plain_mid(shots: int = 128) -> Circuit:
    """n = 1,024, 100 layers, measure all, 128 shots (generator seed 1)."""
    return layered_circuit(1024, 100, shots, gen_seed=1)


def plain_large() -> Circuit:
    """n = 10,000, 20 layers, measure all, 1 shot (generator seed 2)."""
    return layered_circuit(10_000, 20, 1, gen_seed=2)


def plain_xlarge() -> Circuit:
    """n = 25,000, 20 layers, 1 shot (generator seed 6): a tableau of 313 MB,
    larger than the 256 MB Infinity Cache, for the HBM-bound measurement path;
    measured on a prefix of its qubits."""
    return layered_circuit(25_000, 20, 1, gen_seed=6)


def batch_sizes(count: int = 4096, seed: int = 3, n_lo: int = 8, n_hi: int = 256):
    """Sizes of the batched workload: n ~ U{n_lo..n_hi}, depth ~ U{n..4n}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    depths = rng.integers(ns, 4 * ns + 1)
    return ns.astype(np.int64), depths.astype(np.int64)


def batch_circuit(i: int, ns, depths, seed: int = 3, shots: int = 4) -> Circuit:
    """Circuit ``i`` of the batched workload; drawn from its own child stream
    so any subset can be generated independently."""
    n, depth = int(ns[i]), int(depths[i])
    return layered_circuit(n, depth, shots, gen_seed=[seed, 1, i], circuit_id=i)


def batch_workload(count: int = 4096, seed: int = 3, shots: int = 4,
                   n_lo: int = 8, n_hi: int = 256, indices=None):
    """The batched workload (4,096 circuits, 4 shots each) or a subset."""
    ns, depths = batch_sizes(count, seed, n_lo, n_hi)
    idx = range(count) if indices is None else indices
    return [batch_circuit(i, ns, depths, seed, shots) for i in idx]


@dataclasses.dataclass
class Request:
    """One serving request: a circuit plus its arrival time in seconds."""

    arrival: float
    circuit: Circuit


def serving_params(count: int, rate_hz: float, seed: int = 4,
                   n_lo: int = 16, n_hi: int = 4096, shots_hi: int = 1024):
    """Arrival times, sizes and shot counts of the serving workload.

    Poisson arrivals at ``rate_hz``; n log-uniform on [n_lo, n_hi] (the floor of
    exp(U[ln n_lo, ln(n_hi + 1))), clamped to n_hi); depth 2n; shots ~ U{1..shots_hi}.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    u = rng.uniform(math.log(n_lo), math.log(n_hi + 1), size=count)
    ns = np.minimum(np.floor(np.exp(u)).astype(np.int64), n_hi)
    shots = rng.integers(1, shots_hi + 1, size=count)
    return arrivals, ns, shots


def serving_request(i: int, arrivals, ns, shots, seed: int = 4) -> Request:
    n = int(ns[i])
    c = layered_circuit(n, 2 * n, int(shots[i]), gen_seed=[seed, 2, i], circuit_id=i)
    return Request(arrival=float(arrivals[i]), circuit=c)


def serving_workload(count: int, rate_hz: float, seed: int = 4, **kw):
    arrivals, ns, shots = serving_params(count, rate_hz, seed, **kw)
    return [serving_request(i, arrivals, ns, shots, seed) for i in range(count)]


# Gate-list op codes (the library's public numbering).
OP_H, OP_S, OP_CNOT, OP_SDG, OP_X, OP_Y, OP_Z, OP_CZ, OP_SWAP = range(9)
TWO_QUBIT_OPS = (OP_CNOT, OP_CZ, OP_SWAP)


def random_gate_list(rng: np.random.Generator, n: int, count: int, p_cnot: float = 0.4,
                     full: bool = False):
    """Unstructured gate list: op codes 0 = H, 1 = S, 2 = CNOT(a -> b); with
    ``full`` also 3 = S^dagger, 4..6 = X, Y, Z, 7 = CZ, 8 = SWAP (two-qubit ops
    with probability p_cnot, spread evenly over CNOT, CZ and SWAP).  b is 0
    for single-qubit ops."""
    two = rng.random(count) < p_cnot
    if full:
        single = np.array([OP_H, OP_S, OP_SDG, OP_X, OP_Y, OP_Z], np.uint8)
        ops = np.where(two, np.array(TWO_QUBIT_OPS, np.uint8)[rng.integers(0, 3, size=count)],
                       single[rng.integers(0, 6, size=count)]).astype(np.uint8)
    else:
        ops = np.where(two, OP_CNOT, rng.integers(0, 2, size=count)).astype(np.uint8)
    a = rng.integers(0, n, size=count).astype(np.uint32)
    b = rng.integers(0, n - 1, size=count).astype(np.uint32) if n > 1 else np.zeros(count, np.uint32)
    b = np.where(b >= a, b + 1, b).astype(np.uint32)
    is_two = np.isin(ops, TWO_QUBIT_OPS)
    if n == 1:
        ops[:] = np.where(is_two, OP_H, ops)
        is_two[:] = False
    b = np.where(is_two, b, 0).astype(np.uint32)
    return ops, a, b

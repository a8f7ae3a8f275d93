"""CPU oracle for stabilizer-tableau simulation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never links or calls it.

The arithmetic lives in ``chp.c`` (plain C, one byte per tableau bit), built
with gcc into ``oracle/_build/liboracle.so`` by :func:`build`.  This module is
argument marshalling only.  The algorithm is the phase-space tableau method the
paper's Clifford backend implements (Sec. 2, citing Aaronson & Gottesman 2004):
gate rules (H, S, CNOT and the rest of the Clifford gate set: S^dagger, X, Y,
Z, CZ, SWAP), rowsum with the phase function g, and measurement of Z (or X, Y)
on one qubit with a random branch (pivot found) and a deterministic branch
(scratch-row product).

Every function here is pinned by ``tests/test_oracle_*.py`` against brute-force
statevector simulation, explicit Pauli matrices, closed-form identities,
symplectic invariants and numpy's Philox4x64-10.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "chp.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_OUT_DIR, "liboracle.so")
_lib = None

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    """Compile chp.c with gcc -O2 into oracle/_build/liboracle.so."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    lib.orc_new.restype = vp
    lib.orc_new.argtypes = [ctypes.c_int]
    lib.orc_free.argtypes = [vp]
    lib.orc_clone.restype = vp
    lib.orc_clone.argtypes = [vp]
    lib.orc_n.argtypes = [vp]
    lib.orc_anomalies.restype = ctypes.c_long
    lib.orc_anomalies.argtypes = [vp]
    lib.orc_get.argtypes = [vp, _u8p, _u8p, _u8p]
    lib.orc_set.argtypes = [vp, _u8p, _u8p, _u8p]
    for f in (lib.orc_h, lib.orc_s, lib.orc_sdg, lib.orc_x, lib.orc_y, lib.orc_z):
        f.argtypes = [vp, ctypes.c_int]
    for f in (lib.orc_cnot, lib.orc_cz, lib.orc_swap):
        f.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.orc_apply_layers.argtypes = [vp, ctypes.c_int, _u8p, _u8p, _u32p, _u32p, ctypes.c_int]
    lib.orc_apply_gates.restype = ctypes.c_long
    lib.orc_apply_gates.argtypes = [vp, ctypes.c_long, _u8p, _u32p, _u32p]
    lib.orc_reset.argtypes = [vp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                              ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
    lib.orc_measure_pauli.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                      ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.POINTER(ctypes.c_int)]
    lib.orc_g.argtypes = [ctypes.c_int] * 4
    lib.orc_rowsum.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    lib.orc_measure.argtypes = [vp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
    lib.orc_measure_list.argtypes = [vp, ctypes.c_int, _u32p, ctypes.c_uint64, ctypes.c_uint64,
                                     ctypes.c_uint64, ctypes.c_uint64, _u8p, _u8p]
    lib.orc_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
    lib.orc_random_bit.argtypes = [ctypes.c_uint64] * 4
    lib.orc_run_shot.argtypes = [ctypes.c_int, ctypes.c_int, _u8p, _u8p, _u32p, _u32p, ctypes.c_int,
                                 ctypes.c_int, _u32p, ctypes.c_uint64, ctypes.c_uint64,
                                 ctypes.c_uint64, _u8p, _u8p, _u8p, _u8p, _u8p]
    _lib = lib
    return lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


# Gate-list op codes and measurement bases (the same numbering as the library's
# public header, an interface both consume).
GATE_CODES = {"h": 0, "s": 1, "cnot": 2, "sdg": 3, "x": 4, "y": 5, "z": 6, "cz": 7, "swap": 8}
BASIS_Z, BASIS_X, BASIS_Y = 0, 1, 2
# (x, z) bits of the measured Pauli per basis code
_BASIS_BITS = {BASIS_Z: (0, 1), BASIS_X: (1, 0), BASIS_Y: (1, 1)}


def philox4x64_10(counter, key) -> np.ndarray:
    """Raw Philox4x64-10 block for a 4-word counter and 2-word key."""
    lib = _load()
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib.orc_philox4x64_10(_p(c, _u64p), _p(k, _u64p), _p(out, _u64p))
    return out


def random_bit(seed: int, circuit: int, shot: int, m: int) -> int:
    """Outcome bit of a random measurement: Philox key (seed, 0), counter (m, shot, circuit, 0)."""
    return int(_load().orc_random_bit(seed, circuit, shot, m))


def g(x1: int, z1: int, x2: int, z2: int) -> int:
    return int(_load().orc_g(x1, z1, x2, z2))


class Tableau:
    """Byte-per-bit tableau on the host (2n rows + 1 scratch row)."""

    def __init__(self, n: int, _handle=None):
        self._lib = _load()
        self.n = int(n)
        self._h = _handle if _handle is not None else self._lib.orc_new(self.n)
        if not self._h:
            raise MemoryError("oracle tableau allocation failed")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_free(h)
            self._h = None

    def clone(self) -> "Tableau":
        return Tableau(self.n, self._lib.orc_clone(self._h))

    @property
    def anomalies(self) -> int:
        """Rowsums whose sign exponent came out odd where the rows should commute."""
        return int(self._lib.orc_anomalies(self._h))

    def h(self, a: int):
        self._lib.orc_h(self._h, int(a))
        return self

    def s(self, a: int):
        self._lib.orc_s(self._h, int(a))
        return self

    def cnot(self, a: int, b: int):
        self._lib.orc_cnot(self._h, int(a), int(b))
        return self

    def sdg(self, a: int):
        self._lib.orc_sdg(self._h, int(a))
        return self

    def x(self, a: int):
        self._lib.orc_x(self._h, int(a))
        return self

    def y(self, a: int):
        self._lib.orc_y(self._h, int(a))
        return self

    def z(self, a: int):
        self._lib.orc_z(self._h, int(a))
        return self

    def cz(self, a: int, b: int):
        self._lib.orc_cz(self._h, int(a), int(b))
        return self

    def swap(self, a: int, b: int):
        self._lib.orc_swap(self._h, int(a), int(b))
        return self

    def rowsum(self, h: int, i: int) -> int:
        return int(self._lib.orc_rowsum(self._h, int(h), int(i)))

    def apply_layers(self, h, s, ctrl, tgt):
        h = np.ascontiguousarray(h, np.uint8)
        s = np.ascontiguousarray(s, np.uint8)
        ctrl = np.ascontiguousarray(ctrl, np.uint32)
        tgt = np.ascontiguousarray(tgt, np.uint32)
        depth = h.shape[0]
        npairs = ctrl.shape[1] if ctrl.ndim == 2 else 0
        self._lib.orc_apply_layers(self._h, depth, _p(h, _u8p), _p(s, _u8p),
                                   _p(ctrl, _u32p), _p(tgt, _u32p), npairs)
        return self

    def apply_circuit_gates(self, c):
        return self.apply_layers(c.h, c.s, c.ctrl, c.tgt)

    def apply_gates(self, ops, a, b):
        """Gate list with op codes GATE_CODES (H, S, CNOT, SDG, X, Y, Z, CZ, SWAP)."""
        ops = np.ascontiguousarray(ops, np.uint8)
        a = np.ascontiguousarray(a, np.uint32)
        b = np.ascontiguousarray(b, np.uint32)
        bad = self._lib.orc_apply_gates(self._h, len(ops), _p(ops, _u8p), _p(a, _u32p), _p(b, _u32p))
        if bad >= 0:
            raise ValueError("unknown gate op %d at position %d" % (int(ops[bad]), bad))
        return self

    def measure(self, a: int, seed: int = 0, circuit: int = 0, shot: int = 0, m: int = 0):
        """Z-measure qubit a. Returns (outcome, was_random)."""
        kind = ctypes.c_int(0)
        out = self._lib.orc_measure(self._h, int(a), seed, circuit, shot, m, ctypes.byref(kind))
        return int(out), bool(kind.value)

    def measure_pauli(self, a: int, basis: int, seed: int = 0, circuit: int = 0, shot: int = 0,
                      m: int = 0):
        """Measure X (basis 1), Y (2) or Z (0) on qubit a. Returns (outcome, was_random)."""
        px, pz = _BASIS_BITS[int(basis)]
        kind = ctypes.c_int(0)
        out = self._lib.orc_measure_pauli(self._h, int(a), px, pz, seed, circuit, shot, m,
                                          ctypes.byref(kind))
        return int(out), bool(kind.value)

    def reset(self, a: int, seed: int = 0, circuit: int = 0, shot: int = 0, m: int = 0):
        """Reset qubit a to |0> (Z-measure, then X where the outcome was 1).
        Returns (outcome, was_random) of the measurement."""
        kind = ctypes.c_int(0)
        out = self._lib.orc_reset(self._h, int(a), seed, circuit, shot, m, ctypes.byref(kind))
        return int(out), bool(kind.value)

    def pauli(self, a: int, p: int):
        """Apply the Pauli p (1 = X, 2 = Y, 3 = Z; 0 = nothing) to qubit a."""
        if p:
            (self.x, self.y, self.z)[int(p) - 1](a)
        return self

    def measure_bases(self, qubits, bases, seed=0, circuit=0, shot=0, m0=0):
        """measure_pauli over a list, measurement index m0 + position."""
        out = np.zeros(len(qubits), np.uint8)
        kind = np.zeros(len(qubits), np.uint8)
        for i, (q, b) in enumerate(zip(qubits, bases)):
            out[i], kind[i] = self.measure_pauli(int(q), int(b), seed, circuit, shot, m0 + i)
        return out, kind

    def measure_list(self, qubits, seed=0, circuit=0, shot=0, m0=0):
        q = np.ascontiguousarray(qubits, np.uint32)
        out = np.zeros(len(q), np.uint8)
        kind = np.zeros(len(q), np.uint8)
        self._lib.orc_measure_list(self._h, len(q), _p(q, _u32p), seed, circuit, shot, m0,
                                   _p(out, _u8p), _p(kind, _u8p))
        return out, kind

    def get(self):
        """(x, z, r) as uint8 arrays of shape [2n, n], [2n, n], [2n]."""
        n = self.n
        x = np.zeros((2 * n, n), np.uint8)
        z = np.zeros((2 * n, n), np.uint8)
        r = np.zeros(2 * n, np.uint8)
        self._lib.orc_get(self._h, _p(x, _u8p), _p(z, _u8p), _p(r, _u8p))
        return x, z, r

    def set(self, x, z, r):
        n = self.n
        x = np.ascontiguousarray(x, np.uint8).reshape(2 * n, n)
        z = np.ascontiguousarray(z, np.uint8).reshape(2 * n, n)
        r = np.ascontiguousarray(r, np.uint8).reshape(2 * n)
        self._lib.orc_set(self._h, _p(x, _u8p), _p(z, _u8p), _p(r, _u8p))
        return self


def run_shot(c, shot: int, want_tableau: bool = False):
    """Run circuit ``c`` (an ``inputs.Circuit``) for one shot from |0...0>.

    Returns (outcomes uint8[k], kinds uint8[k]) and, if requested, the final
    tableau (x, z, r) of that shot.
    """
    lib = _load()
    n = c.n
    h = np.ascontiguousarray(c.h, np.uint8)
    s = np.ascontiguousarray(c.s, np.uint8)
    ctrl = np.ascontiguousarray(c.ctrl, np.uint32)
    tgt = np.ascontiguousarray(c.tgt, np.uint32)
    q = np.ascontiguousarray(c.qubits, np.uint32)
    k = len(q)
    out = np.zeros(k, np.uint8)
    kind = np.zeros(k, np.uint8)
    if want_tableau:
        x = np.zeros((2 * n, n), np.uint8)
        z = np.zeros((2 * n, n), np.uint8)
        r = np.zeros(2 * n, np.uint8)
        xp, zp, rp = _p(x, _u8p), _p(z, _u8p), _p(r, _u8p)
    else:
        x = z = r = None
        xp = zp = rp = None
    rc = lib.orc_run_shot(n, c.depth, _p(h, _u8p), _p(s, _u8p), _p(ctrl, _u32p), _p(tgt, _u32p),
                          ctrl.shape[1] if ctrl.ndim == 2 else 0, k, _p(q, _u32p),
                          c.seed, c.circuit_id, shot, _p(out, _u8p), _p(kind, _u8p), xp, zp, rp)
    if rc != 0:
        raise MemoryError("oracle run_shot failed")
    if want_tableau:
        return out, kind, (x, z, r)
    return out, kind


def run_circuit(c, shots=None):
    """Outcomes [len(shots), k] for the listed shot indices (default: all)."""
    shots = range(c.shots) if shots is None else shots
    rows = [run_shot(c, int(s))[0] for s in shots]
    return np.stack(rows) if rows else np.zeros((0, len(c.qubits)), np.uint8)


def run_program(prog, shot: int):
    """Run a program of ``inputs.programs`` (mid-circuit measurement, reset,
    conditioned Paulis) for one shot from |0...0>.  Returns (record uint8[M],
    random flags uint8[M], final Tableau)."""
    t = Tableau(prog.n)
    M = prog.measurements
    rec = np.zeros(M, np.uint8)
    kinds = np.zeros(M, np.uint8)
    col = 0
    for st in prog.steps:
        kind = st[0]
        if kind == "gates":
            t.apply_gates(st[1], st[2], st[3])
        elif kind in ("measure", "reset"):
            fn = t.measure if kind == "measure" else t.reset
            for q in st[1]:
                rec[col], kinds[col] = fn(int(q), seed=prog.seed, circuit=prog.circuit_id, shot=shot, m=col)
                col += 1
        elif kind == "cond":
            for q, p, c in zip(st[1], st[2], st[3]):
                if rec[int(c)]:
                    t.pauli(int(q), int(p))
        elif kind == "cgates":
            if rec[int(st[1])]:
                t.apply_gates(st[2], st[3], st[4])
        else:
            raise ValueError("unknown program step %r" % (kind,))
    return rec, kinds, t

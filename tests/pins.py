"""Independent mathematical pins for the tableau oracle (test helpers).

Nothing here uses the tableau method: states are dense 2^n complex vectors and
Pauli operators are explicit matrices.  Qubit j is bit j of the basis index.
"""
from __future__ import annotations

import numpy as np

I2 = np.eye(2, dtype=complex)
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
HM = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
SM = np.array([[1, 0], [0, 1j]], dtype=complex)


def pauli1(x: int, z: int) -> np.ndarray:
    """Single-qubit Pauli for tableau bits (x, z): I, X, Z, Y."""
    return {(0, 0): I2, (1, 0): PX, (0, 1): PZ, (1, 1): PY}[(int(x), int(z))]


def kron_list(mats):
    """Kronecker product with qubit 0 as the least significant index bit."""
    out = np.array([[1.0 + 0j]])
    for m in mats:
        out = np.kron(m, out)
    return out


def pauli_string(x, z, r=0) -> np.ndarray:
    """(-1)^r * tensor_j P(x_j, z_j) as a dense 2^n x 2^n matrix."""
    m = kron_list([pauli1(a, b) for a, b in zip(x, z)])
    return -m if r else m


class StateVector:
    """Dense statevector simulator, n <= ~10."""

    def __init__(self, n: int):
        self.n = n
        self.psi = np.zeros(2 ** n, dtype=complex)
        self.psi[0] = 1.0

    def _apply1(self, u, a):
        psi = self.psi.reshape([2] * self.n)  # axis k <-> qubit n-1-k
        ax = self.n - 1 - a
        psi = np.moveaxis(np.tensordot(u, psi, axes=([1], [ax])), 0, ax)
        self.psi = psi.reshape(-1)

    def h(self, a):
        self._apply1(HM, a)

    def s(self, a):
        self._apply1(SM, a)

    def cnot(self, c, t):
        idx = np.arange(2 ** self.n)
        flip = ((idx >> c) & 1) == 1
        tgt = idx ^ (1 << t)
        new = self.psi.copy()
        new[idx[flip]] = self.psi[tgt[flip]]
        self.psi = new

    def apply_layers(self, h, s, ctrl, tgt):
        for l in range(h.shape[0]):
            for q in range(self.n):
                if h[l, q]:
                    self.h(q)
                if s[l, q]:
                    self.s(q)
            for c, t in zip(ctrl[l], tgt[l]):
                self.cnot(int(c), int(t))

    def sdg(self, a):
        self._apply1(SM.conj(), a)

    def x(self, a):
        self._apply1(PX, a)

    def y(self, a):
        self._apply1(PY, a)

    def z(self, a):
        self._apply1(PZ, a)

    def cz(self, a, b):
        idx = np.arange(2 ** self.n)
        both = (((idx >> a) & 1) & ((idx >> b) & 1)) == 1
        self.psi = np.where(both, -self.psi, self.psi)

    def swap(self, a, b):
        idx = np.arange(2 ** self.n)
        src = idx ^ ((((idx >> a) ^ (idx >> b)) & 1) * ((1 << a) | (1 << b)))
        self.psi = self.psi[src]

    def apply_gates(self, ops, a, b):
        """Op codes: 0 H, 1 S, 2 CNOT(a -> b), 3 S^dagger, 4 X, 5 Y, 6 Z, 7 CZ, 8 SWAP."""
        one = {0: self.h, 1: self.s, 3: self.sdg, 4: self.x, 5: self.y, 6: self.z}
        two = {2: self.cnot, 7: self.cz, 8: self.swap}
        for o, x, y in zip(ops, a, b):
            if int(o) in one:
                one[int(o)](int(x))
            else:
                two[int(o)](int(x), int(y))

    def prob_minus(self, a, pauli) -> float:
        """Probability of eigenvalue -1 when measuring the 2x2 Pauli on qubit a."""
        proj = (I2 - pauli) / 2
        keep = self.psi.copy()
        self._apply1(proj, a)
        p = float(np.linalg.norm(self.psi) ** 2)
        self.psi = keep
        return p

    def collapse_pauli(self, a, pauli, bit):
        """Project onto eigenvalue (-1)^bit of the Pauli on qubit a."""
        self._apply1((I2 + (-1) ** bit * pauli) / 2, a)
        nrm = np.linalg.norm(self.psi)
        assert nrm > 1e-9, "collapse onto a zero-probability outcome"
        self.psi = self.psi / nrm

    def prob_one(self, a) -> float:
        idx = np.arange(2 ** self.n)
        return float(np.sum(np.abs(self.psi[((idx >> a) & 1) == 1]) ** 2))

    def collapse(self, a, bit):
        idx = np.arange(2 ** self.n)
        keep = ((idx >> a) & 1) == bit
        self.psi = np.where(keep, self.psi, 0)
        nrm = np.linalg.norm(self.psi)
        assert nrm > 1e-9, "collapse onto a zero-probability outcome"
        self.psi = self.psi / nrm

    def expect(self, op) -> complex:
        return complex(np.vdot(self.psi, op @ self.psi))

    def support_size(self) -> int:
        return int(np.sum(np.abs(self.psi) ** 2 > 1e-12))


def symplectic_ok(x, z) -> bool:
    """Tableau rows obey <D_i, D_j> = <S_i, S_j> = 0 and <D_i, S_j> = delta_ij
    under the symplectic form <a, b> = x_a . z_b + z_a . x_b (mod 2)."""
    x = x.astype(np.int64)
    z = z.astype(np.int64)
    n = x.shape[1]
    form = (x @ z.T + z @ x.T) % 2
    want = np.zeros((2 * n, 2 * n), np.int64)
    want[np.arange(n), n + np.arange(n)] = 1
    want[n + np.arange(n), np.arange(n)] = 1
    return bool(np.array_equal(form, want))

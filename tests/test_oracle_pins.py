"""Pins for the CPU oracle against mathematics that does not use the tableau method.

Each check targets a part of the oracle where a plausible slip (a dropped sign
term, a swapped operand of g, a wrong pivot row, an off-by-n index) would show:
  * Philox4x64-10 vs numpy's independent implementation and Random123 KATs;
  * g vs explicit 2x2 Pauli products (all 16 cases);
  * H / S / CNOT row updates vs explicit conjugation U P U^dagger;
  * rowsum vs explicit Pauli-string products with the complex phase tracked;
  * closed-form identities (H^2, S^4, S^2 = Z, CNOT^2, (HS)^3) bit-exactly;
  * S^dagger, X, Y, Z, CZ, SWAP row updates vs explicit conjugation, and the
    identities tying them to H / S / CNOT;
  * X-, Y- and Z-basis measurements vs a dense statevector (probabilities and
    collapse), and hand-worked eigenstates of each basis;
  * random circuits with interleaved measurements vs a dense statevector;
  * Bell / GHZ correlations; symplectic invariants; log2 |supp psi|.
"""
import itertools

import numpy as np
import pytest

import oracle
from inputs import layered_circuit, random_gate_list
from pins import (HM, PX, PY, PZ, SM, StateVector, kron_list, pauli1,
                  pauli_string, symplectic_ok)

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


# ------------------------------------------------------------------ Philox ---

def _numpy_philox_block(counter, key):
    # numpy's Philox pre-increments its 256-bit counter before each block, so
    # starting one below the wanted counter yields the block for that counter.
    c = [int(v) for v in counter]
    borrow = 1
    for i in range(4):
        v = c[i] - borrow
        borrow = 1 if v < 0 else 0
        c[i] = v % (1 << 64)
    g = np.random.Philox(key=np.array(key, np.uint64), counter=np.array(c, np.uint64))
    return g.random_raw(4)


def test_philox_known_answers():
    # Random123 known-answer vectors for philox4x64 with 10 rounds
    zero = oracle.philox4x64_10([0, 0, 0, 0], [0, 0])
    assert [int(v) for v in zero] == [0x16554D9ECA36314C, 0xDB20FE9D672D0FDC,
                                      0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]
    pi = oracle.philox4x64_10([0x243F6A8885A308D3, 0x13198A2E03707344,
                               0xA4093822299F31D0, 0x082EFA98EC4E6C89],
                              [0x452821E638D01377, 0xBE5466CF34E90C6C])
    assert [int(v) for v in pi] == [0xA528F45403E61D95, 0x38C72DBD566E9788,
                                    0xA5A1610E72FD18B5, 0x57BD43B5E52B7FE6]


def test_philox_matches_numpy():
    rng = np.random.default_rng(123)
    for _ in range(200):
        ctr = rng.integers(0, 2 ** 63, size=4, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 4, dtype=np.uint64)
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64) * np.uint64(2)
        ours = oracle.philox4x64_10(ctr, key)
        ref = _numpy_philox_block(ctr, key)
        assert np.array_equal(ours, ref)


def test_random_bit_keying():
    seed, circ, shot, m = 0x240800384, 7, 3, 11
    block = _numpy_philox_block([m, shot, circ, 0], [seed, 0])
    assert oracle.random_bit(seed, circ, shot, m) == int(block[0]) & 1
    bits = [oracle.random_bit(seed, 0, 0, m) for m in range(4000)]
    assert 1800 < sum(bits) < 2200  # a fair coin, loosely


# ----------------------------------------------------------------------- g ---

def test_g_all_sixteen_cases():
    for x1, z1, x2, z2 in itertools.product((0, 1), repeat=4):
        prod = pauli1(x1, z1) @ pauli1(x2, z2)
        res = pauli1(x1 ^ x2, z1 ^ z2)
        k = oracle.g(x1, z1, x2, z2)
        assert np.allclose(prod, (1j ** k) * res), (x1, z1, x2, z2, k)
        assert -1 <= k <= 1


# ------------------------------------------------------------- gate rules ---

def _single_row_tableau(n, x, z, r):
    """Tableau whose row 0 is the given Pauli; other rows are unused filler."""
    t = oracle.Tableau(n)
    X, Z, R = t.get()
    X[0], Z[0], R[0] = x, z, r
    t.set(X, Z, R)
    return t


def _conj_check(n, gate_fn, U):
    for bits in itertools.product((0, 1), repeat=2 * n + 1):
        x = np.array(bits[:n], np.uint8)
        z = np.array(bits[n:2 * n], np.uint8)
        r = bits[2 * n]
        t = _single_row_tableau(n, x, z, r)
        gate_fn(t)
        X, Z, R = t.get()
        want = U @ pauli_string(x, z, r) @ U.conj().T
        got = pauli_string(X[0], Z[0], R[0])
        assert np.allclose(want, got), (x, z, r)


def test_h_rule():
    _conj_check(1, lambda t: t.h(0), HM)


def test_s_rule():
    _conj_check(1, lambda t: t.s(0), SM)


def test_sdg_and_pauli_rules():
    _conj_check(1, lambda t: t.sdg(0), SM.conj())
    _conj_check(1, lambda t: t.x(0), PX)
    _conj_check(1, lambda t: t.y(0), PY)
    _conj_check(1, lambda t: t.z(0), PZ)


def test_cz_and_swap_rules_both_orientations():
    CZ = np.diag([1, 1, 1, -1]).astype(complex)
    SW = np.zeros((4, 4), complex)
    for i in range(4):
        SW[((i & 1) << 1) | (i >> 1), i] = 1
    for a, b in ((0, 1), (1, 0)):
        _conj_check(2, lambda t: t.cz(a, b), CZ)
        _conj_check(2, lambda t: t.swap(a, b), SW)
    # on a third qubit the gate must leave the other column alone
    _conj_check(3, lambda t: t.cz(2, 0), np.diag([1, 1, 1, 1, 1, -1, 1, -1]).astype(complex))


def test_cnot_rule_both_orientations():
    # basis index bit j = qubit j; CNOT(control c, target t)
    def cnot_matrix(c, tq):
        U = np.zeros((4, 4), complex)
        for i in range(4):
            j = i ^ (1 << tq) if (i >> c) & 1 else i
            U[j, i] = 1
        return U
    _conj_check(2, lambda t: t.cnot(0, 1), cnot_matrix(0, 1))
    _conj_check(2, lambda t: t.cnot(1, 0), cnot_matrix(1, 0))


# ------------------------------------------------------------------ rowsum ---

@pytest.mark.parametrize("n", [1, 2, 5, 17, 64])
def test_rowsum_vs_pauli_products(n):
    rng = np.random.default_rng(n)
    for _ in range(60):
        # two random commuting Pauli strings: draw, then fix commutation by
        # flipping one z bit where the first string has an x
        x1, z1 = rng.integers(0, 2, n), rng.integers(0, 2, n)
        x2, z2 = rng.integers(0, 2, n), rng.integers(0, 2, n)
        r1, r2 = int(rng.integers(0, 2)), int(rng.integers(0, 2))
        sym = int((x1 @ z2 + z1 @ x2) % 2)
        if sym:
            j = int(np.flatnonzero(x1 | z1)[0]) if np.any(x1 | z1) else None
            if j is None:
                continue
            if x1[j]:
                z2[j] ^= 1
            else:
                x2[j] ^= 1
        assert int((x1 @ z2 + z1 @ x2) % 2) == 0
        # explicit product phase: (-1)^r1 P1 * (-1)^r2 P2 per qubit with 2x2 matrices
        phase = (-1) ** (r1 + r2) + 0j
        for j in range(n):
            prod = pauli1(x1[j], z1[j]) @ pauli1(x2[j], z2[j])
            res = pauli1(x1[j] ^ x2[j], z1[j] ^ z2[j])
            k = [c for c in range(4) if np.allclose(prod, (1j ** c) * res)]
            assert len(k) == 1
            phase *= 1j ** k[0]
        assert np.isclose(phase.imag, 0) and np.isclose(abs(phase.real), 1)
        want_r = 0 if phase.real > 0 else 1

        t = oracle.Tableau(n)
        X, Z, R = t.get()
        X[0], Z[0], R[0] = x2, z2, r2   # h = 0 (target)
        X[1], Z[1], R[1] = x1, z1, r1   # i = 1 (source): row0 <- row1 * row0
        t.set(X, Z, R)
        e = t.rowsum(0, 1)
        X2, Z2, R2 = t.get()
        assert e in (0, 2)
        assert R2[0] == want_r
        assert np.array_equal(X2[0], x1 ^ x2) and np.array_equal(Z2[0], z1 ^ z2)
        assert np.array_equal(X2[1], x1) and R2[1] == r1


# -------------------------------------------------------------- identities ---

def _random_state(n, seed):
    c = layered_circuit(n, 6, 1, gen_seed=seed)
    t = oracle.Tableau(n)
    t.apply_circuit_gates(c)
    return t


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_identities_bit_exact(seed):
    n = 9
    t = _random_state(n, seed)
    base = t.get()
    for a in range(n):
        for seq in (["h", "h"], ["s"] * 4, ["h", "s"] * 3):
            u = t.clone()
            for gname in seq:
                getattr(u, gname)(a)
            for A, B in zip(u.get(), base):
                assert np.array_equal(A, B), (a, seq)
        u = t.clone().s(a).s(a)
        X, Z, R = u.get()
        assert np.array_equal(X, base[0]) and np.array_equal(Z, base[1])
        assert np.array_equal(R, base[2] ^ base[0][:, a])  # S^2 = Z flips rows with x_a
    for a in range(n):
        for b in range(n):
            if a != b:
                u = t.clone().cnot(a, b).cnot(a, b)
                for A, B in zip(u.get(), base):
                    assert np.array_equal(A, B)


def _same(u, v):
    return all(np.array_equal(A, B) for A, B in zip(u.get(), v.get()))


@pytest.mark.parametrize("seed", [0, 1])
def test_full_gate_set_identities_bit_exact(seed):
    n = 7
    t = _random_state(n, seed)
    for a in range(n):
        assert _same(t.clone().s(a).sdg(a), t)
        assert _same(t.clone().sdg(a).sdg(a), t.clone().z(a))             # S^dagger^2 = Z
        assert _same(t.clone().h(a).z(a).h(a), t.clone().x(a))            # HZH = X
        assert _same(t.clone().x(a).z(a), t.clone().y(a))                 # Y = i X Z
        for p in ("x", "y", "z"):
            u = t.clone()
            getattr(getattr(u, p)(a), p)(a)
            assert _same(u, t)
    for a in range(n):
        for b in range(n):
            if a == b:
                continue
            assert _same(t.clone().cz(a, b), t.clone().cz(b, a))
            assert _same(t.clone().cz(a, b), t.clone().h(b).cnot(a, b).h(b))
            assert _same(t.clone().swap(a, b), t.clone().cnot(a, b).cnot(b, a).cnot(a, b))
            assert _same(t.clone().cz(a, b).cz(a, b), t)
            assert _same(t.clone().swap(a, b).swap(a, b), t)
    ops, qa, qb = random_gate_list(np.random.default_rng(seed), n, 40, full=True)
    u = t.clone().apply_gates(ops, qa, qb)
    v = t.clone()
    name = {0: "h", 1: "s", 2: "cnot", 3: "sdg", 4: "x", 5: "y", 6: "z", 7: "cz", 8: "swap"}
    for o, x, y in zip(ops, qa, qb):
        f = getattr(v, name[int(o)])
        f(int(x), int(y)) if int(o) in (2, 7, 8) else f(int(x))
    assert _same(u, v)
    with pytest.raises(ValueError):
        t.clone().apply_gates([9], [0], [0])


# ------------------------------------------------------- vs a statevector ---

def _check_stabilizers(t, sv):
    X, Z, R = t.get()
    n = t.n
    for i in range(n, 2 * n):
        v = sv.expect(pauli_string(X[i], Z[i], R[i]))
        assert np.isclose(v, 1.0, atol=1e-9), (i, v)
    assert symplectic_ok(X, Z)


@pytest.mark.parametrize("seed", range(12))
def test_random_circuits_with_measurements_vs_statevector(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(1, 8))
    t = oracle.Tableau(n)
    sv = StateVector(n)
    m = 0
    for block in range(6):
        ops, a, b = random_gate_list(rng, n, int(rng.integers(1, 15)))
        t.apply_gates(ops, a, b)
        sv.apply_gates(ops, a, b)
        _check_stabilizers(t, sv)
        for _ in range(int(rng.integers(0, 3))):
            q = int(rng.integers(0, n))
            p1 = sv.prob_one(q)
            bit, rnd = t.measure(q, seed=99, circuit=seed, shot=0, m=m)
            if rnd:
                assert np.isclose(p1, 0.5, atol=1e-9)
                assert bit == oracle.random_bit(99, seed, 0, m)
            else:
                assert np.isclose(p1, float(bit), atol=1e-9)
            sv.collapse(q, bit)
            m += 1
            _check_stabilizers(t, sv)
    assert t.anomalies == 0


@pytest.mark.parametrize("seed", range(10))
def test_full_gate_set_and_pauli_measurements_vs_statevector(seed):
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(1, 7))
    t = oracle.Tableau(n)
    sv = StateVector(n)
    mats = {oracle.BASIS_Z: PZ, oracle.BASIS_X: PX, oracle.BASIS_Y: PY}
    m = 0
    for block in range(6):
        ops, a, b = random_gate_list(rng, n, int(rng.integers(1, 15)), full=True)
        t.apply_gates(ops, a, b)
        sv.apply_gates(ops, a, b)
        _check_stabilizers(t, sv)
        for _ in range(int(rng.integers(0, 4))):
            q = int(rng.integers(0, n))
            basis = int(rng.integers(0, 3))
            p1 = sv.prob_minus(q, mats[basis])
            bit, rnd = t.measure_pauli(q, basis, seed=98, circuit=seed, shot=0, m=m)
            if rnd:
                assert np.isclose(p1, 0.5, atol=1e-9)
                assert bit == oracle.random_bit(98, seed, 0, m)
            else:
                assert np.isclose(p1, float(bit), atol=1e-9), (basis, p1, bit)
            sv.collapse_pauli(q, mats[basis], bit)
            m += 1
            _check_stabilizers(t, sv)
    assert t.anomalies == 0


def test_pauli_measurement_eigenstates():
    """Eigenstates of each basis measure deterministically with the right sign;
    the other two bases are random on them and leave +-P_a in the stabilizer."""
    X_, Y_, Z_ = oracle.BASIS_X, oracle.BASIS_Y, oracle.BASIS_Z
    cases = [  # (preparation, basis, outcome)
        (lambda t: t, Z_, 0), (lambda t: t.x(0), Z_, 1),
        (lambda t: t.h(0), X_, 0), (lambda t: t.x(0).h(0), X_, 1),
        (lambda t: t.h(0).s(0), Y_, 0), (lambda t: t.h(0).sdg(0), Y_, 1),
    ]
    for prep, basis, want in cases:
        assert prep(oracle.Tableau(1)).measure_pauli(0, basis) == (want, False)
        for other in {X_, Y_, Z_} - {basis}:
            t = prep(oracle.Tableau(1))
            bit, rnd = t.measure_pauli(0, other, seed=6, m=1)
            assert rnd and bit == oracle.random_bit(6, 0, 0, 1)
            X, Z, R = t.get()
            px, pz = {X_: (1, 0), Y_: (1, 1), Z_: (0, 1)}[other]
            assert (X[1, 0], Z[1, 0], R[1]) == (px, pz, bit)
            assert t.measure_pauli(0, other, m=2) == (bit, False)


@pytest.mark.parametrize("n", [3, 6, 10])
def test_measure_all_random_count_is_log_support(n):
    for seed in range(4):
        c = layered_circuit(n, 5, 1, gen_seed=[n, seed])
        t = oracle.Tableau(n).apply_circuit_gates(c)
        sv = StateVector(n)
        sv.apply_layers(c.h, c.s, c.ctrl, c.tgt)
        _check_stabilizers(t, sv)
        supp = sv.support_size()
        out, kinds = t.measure_list(np.arange(n), seed=5, circuit=seed)
        assert 2 ** int(kinds.sum()) == supp
        # the outcome string lies in the support of the state
        idx = int(sum(int(b) << j for j, b in enumerate(out)))
        assert abs(sv.psi[idx]) > 1e-9
        assert t.anomalies == 0


def test_bell_and_ghz():
    for shot in range(20):
        t = oracle.Tableau(2).h(0).cnot(0, 1)
        b0, r0 = t.measure(0, seed=1, shot=shot, m=0)
        b1, r1 = t.measure(1, seed=1, shot=shot, m=1)
        assert r0 and not r1 and b0 == b1
    outs = set()
    for shot in range(32):
        n = 12
        t = oracle.Tableau(n).h(0)
        for q in range(1, n):
            t.cnot(q - 1, q)
        out, kinds = t.measure_list(np.arange(n), seed=3, shot=shot)
        assert kinds[0] == 1 and kinds[1:].sum() == 0
        assert len(set(out.tolist())) == 1
        outs.add(int(out[0]))
    assert outs == {0, 1}


def test_plus_state_measured_twice_and_zero_state():
    t = oracle.Tableau(1).h(0)
    b0, r0 = t.measure(0, seed=4, m=0)
    b1, r1 = t.measure(0, seed=4, m=1)
    assert r0 and not r1 and b0 == b1
    t = oracle.Tableau(7)
    out, kinds = t.measure_list(np.arange(7))
    assert out.sum() == 0 and kinds.sum() == 0
    # |1> via H S S H = X: deterministic 1
    t = oracle.Tableau(1).h(0).s(0).s(0).h(0)
    assert t.measure(0) == (1, False)


def test_symplectic_invariants_after_measurements():
    n = 40
    c = layered_circuit(n, 8, 1, gen_seed=77)
    t = oracle.Tableau(n).apply_circuit_gates(c)
    X, Z, _ = t.get()
    assert symplectic_ok(X, Z)
    for k in range(0, n, 3):
        t.measure(k, m=k)
        X, Z, _ = t.get()
        assert symplectic_ok(X, Z)
    assert t.anomalies == 0


@pytest.mark.parametrize("n", [7, 200, 201])
def test_layer_routine_equals_gate_by_gate(n):
    """The oracle's layer routine (every rule applied row by row, all gates of
    a layer per row) against its gate-by-gate routine on the same circuit
    written out as a gate list (per layer: H then S on each qubit, then the
    layer's CNOTs): identical tableaux, signs included, after many layers.
    Gates of one layer act on distinct qubits, and each rule touches only its
    own row, so the two orders must agree bit for bit."""
    from inputs import OP_CNOT, OP_H, OP_S
    c = layered_circuit(n, 30, 1, gen_seed=[90, n])
    ops, qa, qb = [], [], []
    for layer in range(c.depth):
        for q in range(n):
            if c.h[layer, q]:
                ops.append(OP_H); qa.append(q); qb.append(0)
            if c.s[layer, q]:
                ops.append(OP_S); qa.append(q); qb.append(0)
        for a_, b_ in zip(c.ctrl[layer], c.tgt[layer]):
            ops.append(OP_CNOT); qa.append(int(a_)); qb.append(int(b_))
    by_layers = oracle.Tableau(n).apply_circuit_gates(c).get()
    by_gates = oracle.Tableau(n).apply_gates(np.array(ops, np.uint8), np.array(qa, np.uint32),
                                             np.array(qb, np.uint32)).get()
    for A, B in zip(by_layers, by_gates):
        assert np.array_equal(A, B)
    # a planted mistake fails the comparison: S before H on one qubit of the
    # first layer that has both
    both = np.flatnonzero(c.h[0] & c.s[0])
    assert len(both)
    j = ops.index(OP_H, 0)
    while qa[j] != both[0] or ops[j] != OP_H:
        j += 1
    ops[j], ops[j + 1] = ops[j + 1], ops[j]
    planted = oracle.Tableau(n).apply_gates(np.array(ops, np.uint8), np.array(qa, np.uint32),
                                            np.array(qb, np.uint32)).get()
    assert any(not np.array_equal(A, B) for A, B in zip(by_layers, planted))


def test_run_shot_matches_stepwise():
    c = layered_circuit(20, 10, 3, gen_seed=5, circuit_id=4)
    for shot in range(3):
        out, kind, (x, z, r) = oracle.run_shot(c, shot, want_tableau=True)
        t = oracle.Tableau(20).apply_circuit_gates(c)
        o2, k2 = t.measure_list(c.qubits, seed=c.seed, circuit=4, shot=shot)
        assert np.array_equal(out, o2) and np.array_equal(kind, k2)
        for A, B in zip((x, z, r), t.get()):
            assert np.array_equal(A, B)


def test_hand_worked_pivot_example():
    """Worked by hand from the gate rules and the smallest-pivot reading.

    n = 2, circuit H(0) H(1) CNOT(0 -> 1) gives rows
      0: Z0   1: Z0 Z1   2: X0 X1   3: X1          (all signs +)
    Measuring qubit 1: stabilizer rows 2 and 3 both have x_1 = 1, so p = 2.
    Row 3 <- row 2 * row 3 = X0 (sign +), row 0 <- old row 2 = X0 X1, and
    row 2 <- (-1)^b Z1 with b the Philox bit.  A largest-pivot choice would
    instead leave rows 0..3 = Z0, X1, X0, Z1.
    """
    t = oracle.Tableau(2).h(0).h(1).cnot(0, 1)
    X, Z, R = t.get()
    assert X.tolist() == [[0, 0], [0, 0], [1, 1], [0, 1]]
    assert Z.tolist() == [[1, 0], [1, 1], [0, 0], [0, 0]]
    assert R.tolist() == [0, 0, 0, 0]
    bit, rnd = t.measure(1, seed=11, circuit=2, shot=5, m=3)
    assert rnd and bit == oracle.random_bit(11, 2, 5, 3)
    X, Z, R = t.get()
    assert X.tolist() == [[1, 1], [0, 0], [0, 0], [1, 0]]
    assert Z.tolist() == [[0, 0], [1, 1], [0, 1], [0, 0]]
    assert R.tolist() == [0, 0, bit, 0]


def test_hand_worked_deterministic_sign():
    """Worked by hand: on |0> the stabilizer is +Z.  H maps it to +X and S
    maps X to +Y; a further H maps Y to -Y, and S maps -Y to +X.  H S S H
    (X up to phase) maps +Z to -Z, so |1> measures 1 deterministically."""
    t = oracle.Tableau(1).h(0).s(0)
    X, Z, R = t.get()
    assert (X[1, 0], Z[1, 0], R[1]) == (1, 1, 0)        # +Y
    t.h(0)
    X, Z, R = t.get()
    assert (X[1, 0], Z[1, 0], R[1]) == (1, 1, 1)        # -Y
    t.s(0)
    X, Z, R = t.get()
    assert (X[1, 0], Z[1, 0], R[1]) == (1, 0, 0)        # +X
    u = oracle.Tableau(1).h(0).s(0).s(0).h(0)
    X, Z, R = u.get()
    assert (X[1, 0], Z[1, 0], R[1]) == (0, 1, 1)        # -Z
    assert u.measure(0) == (1, False)


# ------------------------------------ mid-circuit measurement, reset, feedback ---

def _program_vs_statevector(prog, shot):
    """Replay a program on a dense statevector with the oracle's recorded
    outcomes: each outcome must be possible (and forced when the oracle calls
    it deterministic), and the oracle's stabilizers must hold after every step."""
    from inputs import OP_CNOT, OP_CZ, OP_SWAP  # noqa: F401
    t = oracle.Tableau(prog.n)
    sv = StateVector(prog.n)
    rec = []
    for st in prog.steps:
        if st[0] == "gates":
            t.apply_gates(st[1], st[2], st[3])
            sv.apply_gates(st[1], st[2], st[3])
        elif st[0] in ("measure", "reset"):
            for q in st[1]:
                q = int(q)
                p1 = sv.prob_one(q)
                m = len(rec)
                fn = t.measure if st[0] == "measure" else t.reset
                bit, rnd = fn(q, seed=prog.seed, circuit=prog.circuit_id, shot=shot, m=m)
                if rnd:
                    assert np.isclose(p1, 0.5, atol=1e-9)
                else:
                    assert np.isclose(p1, float(bit), atol=1e-9)
                sv.collapse(q, bit)
                if st[0] == "reset" and bit:
                    sv.x(q)
                if st[0] == "reset":
                    assert np.isclose(sv.prob_one(q), 0.0, atol=1e-9)
                rec.append(bit)
        elif st[0] == "cgates":
            if rec[int(st[1])]:
                t.apply_gates(st[2], st[3], st[4])
                sv.apply_gates(st[2], st[3], st[4])
        else:
            for q, p, c in zip(st[1], st[2], st[3]):
                if rec[int(c)]:
                    (sv.x, sv.y, sv.z)[int(p) - 1](int(q))
                    t.pauli(int(q), int(p))
        _check_stabilizers(t, sv)
    assert t.anomalies == 0
    want, _, u = oracle.run_program(prog, shot)
    assert np.array_equal(want, np.array(rec, np.uint8))
    for A, B in zip(u.get(), t.get()):
        assert np.array_equal(A, B)


@pytest.mark.parametrize("seed", range(8))
def test_programs_with_reset_and_feedback_vs_statevector(seed):
    from inputs import random_program
    n = 1 + seed % 5
    prog = random_program(n, 8, 2, [30, seed], circuit_id=seed)
    kinds = {st[0] for st in prog.steps}
    assert "gates" in kinds
    for shot in range(2):
        _program_vs_statevector(prog, shot)


@pytest.mark.parametrize("seed", range(6))
def test_programs_with_conditioned_gates_vs_statevector(seed):
    from inputs import random_program
    n = 2 + seed % 4
    prog = random_program(n, 12, 3, [32, seed], circuit_id=seed, conditioned_gates=True)
    assert any(st[0] == "cgates" for st in prog.steps)
    for shot in range(3):
        _program_vs_statevector(prog, shot)


def test_reset_returns_zero_state_and_keeps_others():
    """Reset of one half of a Bell pair: the outcome is random, the reset
    qubit is |0> afterwards and the other qubit keeps the measured value."""
    for shot in range(16):
        t = oracle.Tableau(2).h(0).cnot(0, 1)
        bit, rnd = t.reset(0, seed=4, shot=shot, m=0)
        assert rnd and bit == oracle.random_bit(4, 0, shot, 0)
        assert t.measure(0, m=1) == (0, False)
        assert t.measure(1, m=2) == (bit, False)


def test_teleportation_with_conditioned_paulis():
    """Teleport each of the six single-qubit stabilizer states: Bell pair on
    qubits 1, 2; Bell measurement of 0, 1; X on 2 if the outcome of qubit 1
    is 1, Z on 2 if that of qubit 0 is 1.  Qubit 2 then measures
    deterministically in the prepared state's basis with its eigenvalue."""
    from inputs.programs import Program
    from inputs import OP_CNOT, OP_H, OP_S, OP_SDG, OP_X
    Z_, X_, Y_ = oracle.BASIS_Z, oracle.BASIS_X, oracle.BASIS_Y
    preps = [([], Z_, 0), ([OP_X], Z_, 1), ([OP_H], X_, 0), ([OP_X, OP_H], X_, 1),
             ([OP_H, OP_S], Y_, 0), ([OP_H, OP_SDG], Y_, 1)]
    seen = set()
    for ops, basis, want in preps:
        steps = [("gates", np.array(ops + [OP_H, OP_CNOT, OP_CNOT, OP_H], np.uint8),
                  np.array([0] * len(ops) + [1, 1, 0, 0], np.uint32),
                  np.array([0] * len(ops) + [0, 2, 1, 0], np.uint32)),
                 ("measure", np.array([0, 1], np.uint32)),
                 ("cond", np.array([2, 2], np.uint32), np.array([1, 3], np.uint8), np.array([1, 0], np.uint32))]
        prog = Program(n=3, steps=steps, shots=8)
        for shot in range(8):
            rec, kinds, t = oracle.run_program(prog, shot)
            assert kinds.tolist() == [1, 1]
            seen.add(tuple(rec.tolist()))
            assert t.measure_pauli(2, basis, m=9) == (want, False)
    assert len(seen) == 4          # all four Bell outcomes occurred

"""Pins for the uniform-Clifford circuit sampler (inputs.bm_clifford).

Uniformity is checked exactly, not statistically, where the group is small
enough to enumerate: every choice the sampler can make is built and run
through the oracle from |0...0> (whose tableau after a circuit holds the
images of X_i and Z_i, i.e. the Clifford operator itself up to a global
phase).  For n <= 3 the products of all canonical forms must hit every
element of Sp(2n, 2) exactly once; for n <= 2 with signs every element of the
Clifford group exactly once, each with the same probability.  The Mallows
weights are checked against the free-gate counts for n <= 4, and the random
draws statistically.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from inputs.bm_clifford import (clifford_from_choices, draw_k, free_gates, mallows_from_ks,
                                permutation_swaps, random_clifford, round_robin)
from pins import symplectic_ok


def _sp_order(n):
    return 2 ** (n * n) * math.prod(4 ** i - 1 for i in range(1, n + 1))


def _all_ks(n):
    return itertools.product(*[range(1, 2 * (n - a) + 1) for a in range(n)])


def _free_count(h, tau):
    s_free, cz_free, cx_free = free_gates(h, tau)
    return int(s_free.sum()) + int(cz_free.sum()) // 2 + int(cx_free.sum()) // 2


def _tableau(c):
    return oracle.Tableau(c.n).apply_gates(c.ops, c.a, c.b).get()


def _zero_bits(n):
    return (np.zeros((n, n), bool), np.zeros(n, bool), np.zeros((n, n), bool))


def _gate_slots(n, free=None):
    """(kind, i, j) for every gate of a Hadamard-free part (restricted to a
    free set if given): kind 0 CNOT (i < j), 1 S, 2 CZ at the round-robin
    orientation."""
    slots = []
    for first, second in round_robin(n):
        for f, s in zip(first, second):
            lo, hi = min(f, s), max(f, s)
            if free is None or free[2][lo, hi]:
                slots.append((0, lo, hi))
    for q in range(n):
        if free is None or free[0][q]:
            slots.append((1, q, q))
    for first, second in round_robin(n):
        for f, s in zip(first, second):
            if free is None or free[1][f, s]:
                slots.append((2, int(f), int(s)))
    return slots


def _bits_from(n, slots, mask):
    cx, s, cz = _zero_bits(n)
    for (kind, i, j), on in zip(slots, mask):
        if on:
            if kind == 0:
                cx[i, j] = True
            elif kind == 1:
                s[i] = True
            else:
                cz[i, j] = True
    return cx, s, cz


@pytest.mark.parametrize("n", range(1, 10))
def test_round_robin_visits_every_pair_once(n):
    seen = set()
    for first, second in round_robin(n):
        members = list(first) + list(second)
        assert len(set(members)) == len(members)
        for f, s in zip(first, second):
            pair = (min(f, s), max(f, s))
            assert pair not in seen and f != s
            seen.add(pair)
    assert len(seen) == n * (n - 1) // 2


@pytest.mark.parametrize("seed", range(8))
def test_permutation_swaps_move_every_state(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 15))
    tau = rng.permutation(n)
    where = list(range(n))            # where[q] = state held by qubit q
    for layer in permutation_swaps(tau):
        used = [q for pair in layer for q in pair]
        assert len(set(used)) == len(used)
        for x, y in layer:
            where[x], where[y] = where[y], where[x]
    for a in range(n):
        assert where[tau[a]] == a


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_mallows_weights_are_free_gate_counts(n):
    """Every draw sequence gives a distinct (h, tau) (2^n n! of them: the
    signed permutations), its weight prod 2^(k-1) is 2^(number of free
    gates), and the weights sum to prod (4^m - 1) = |Sp(2n, 2)| / |B|."""
    seen = set()
    total = 0
    for ks in _all_ks(n):
        h, tau = mallows_from_ks(ks)
        key = (tuple(h), tuple(tau))
        assert key not in seen
        seen.add(key)
        w = math.prod(2 ** (k - 1) for k in ks)
        assert w == 2 ** _free_count(h, tau), (ks, h, tau)
        total += w
    assert len(seen) == 2 ** n * math.factorial(n)
    assert total == math.prod(4 ** m - 1 for m in range(1, n + 1))
    assert total * 2 ** (n * n) == _sp_order(n)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_canonical_forms_cover_the_symplectic_group_once(n):
    """F2 W F1 over every W, every free-gate subset F1 and every gate subset
    F2 of B: all products distinct and |Sp(2n, 2)| of them."""
    zeros = _zero_bits(n)
    identity_ks = [1] * n
    # x/z part of the tableau as row bitmasks (2n rows of 2n bits)
    def rows(c):
        x, z, _ = _tableau(c)
        return np.array([int("".join(map(str, np.concatenate([x[i], z[i]])[::-1])), 2)
                         for i in range(2 * n)], np.int64)

    wf1 = []
    for ks in _all_ks(n):
        h, tau = mallows_from_ks(ks)
        free = free_gates(h, tau)
        slots = _gate_slots(n, free)
        for mask in itertools.product((0, 1), repeat=len(slots)):
            c = clifford_from_choices(n, ks, zeros, _bits_from(n, slots, mask), np.zeros(n, int))
            wf1.append(rows(c))
    f2_slots = _gate_slots(n)
    f2 = []
    for mask in itertools.product((0, 1), repeat=len(f2_slots)):
        c = clifford_from_choices(n, identity_ks, _bits_from(n, f2_slots, mask), zeros, np.zeros(n, int))
        f2.append(rows(c))
    assert len(f2) == 2 ** (n * n)
    assert len(wf1) * len(f2) == _sp_order(n)
    f2 = np.array(f2)                      # [#F2, 2n] row masks
    keys = []
    for m in wf1:
        # (F2 @ M) row i = xor of M's rows selected by F2's row i bits
        prod = np.zeros(f2.shape, np.int64)
        for j in range(2 * n):
            sel = (f2 >> j) & 1
            prod ^= sel * m[j]
        key = np.zeros(len(f2), np.int64)
        for i in range(2 * n):
            key = (key << (2 * n)) | prod[:, i]
        keys.append(key)
    keys = np.concatenate(keys)
    assert len(np.unique(keys)) == _sp_order(n)


@pytest.mark.parametrize("n", [1, 2])
def test_clifford_group_uniform_with_signs(n):
    """Every choice of the sampler (with its exact probability) yields a
    distinct signed tableau, |Sp(2n, 2)| 4^n of them, all equally likely."""
    f2_slots = _gate_slots(n)
    zeros = _zero_bits(n)
    probs = {}
    for ks in _all_ks(n):
        p_ks = Fraction(math.prod(2 ** (k - 1) for k in ks),
                        math.prod(4 ** m - 1 for m in range(1, n + 1)))
        h, tau = mallows_from_ks(ks)
        f1_slots = _gate_slots(n, free_gates(h, tau))
        for m2 in itertools.product((0, 1), repeat=len(f2_slots)):
            f2 = _bits_from(n, f2_slots, m2)
            for m1 in itertools.product((0, 1), repeat=len(f1_slots)):
                f1 = _bits_from(n, f1_slots, m1)
                for pauli in itertools.product(range(4), repeat=n):
                    c = clifford_from_choices(n, ks, f2, f1, np.array(pauli))
                    x, z, r = _tableau(c)
                    key = (x.tobytes(), z.tobytes(), r.tobytes())
                    assert key not in probs
                    probs[key] = p_ks / 2 ** len(f2_slots) / 2 ** len(f1_slots) / 4 ** n
    assert len(probs) == _sp_order(n) * 4 ** n
    assert set(probs.values()) == {Fraction(1, _sp_order(n) * 4 ** n)}


@pytest.mark.parametrize("m", [1, 2, 3])
def test_draw_k_distribution(m):
    rng = np.random.default_rng(100 + m)
    N = 20000
    counts = np.bincount([draw_k(rng, m) for _ in range(N)], minlength=2 * m + 1)[1:]
    p = np.array([2.0 ** (k - 1) for k in range(1, 2 * m + 1)]) / (4 ** m - 1)
    chi2 = float(((counts - N * p) ** 2 / (N * p)).sum())
    from scipy.stats import chi2 as chi2_dist
    assert chi2_dist.sf(chi2, 2 * m - 1) > 1e-4, (counts, N * p)


def test_random_path_uniform_on_one_qubit():
    """End to end through the random draws: 24 single-qubit Cliffords (with
    signs) equally often."""
    N = 4800
    counts = {}
    for i in range(N):
        x, z, r = _tableau(random_clifford(1, [9, i]))
        key = (x.tobytes(), z.tobytes(), r.tobytes())
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 24
    from scipy.stats import chisquare
    assert chisquare(list(counts.values())).pvalue > 1e-4


@pytest.mark.parametrize("n", [5, 40, 129])
def test_circuit_shape_and_validity(n):
    c = random_clifford(n, [5, n, 0])
    two = np.isin(c.ops, [2, 7, 8])
    assert np.all(c.a < n) and np.all(c.b[two] < n) and np.all(c.a[two] != c.b[two])
    assert np.all(c.b[~two] == 0)
    # about n^2 gates: F2 has ~n(n-1)/2 two-qubit gates, F1 up to as many
    assert 0.3 * n * n < c.gate_count() < 1.3 * n * n + 4 * n
    x, z, _ = _tableau(c)
    assert symplectic_ok(x, z)

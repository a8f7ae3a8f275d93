"""Host logic of the batched path (no GPU): the autotuner's choice of bucket
edges, and the tuning table BatchPlan reads."""
import itertools
import json

import pytest

from paper_2408_00384_amd import autotune as A
from paper_2408_00384_amd import batch as BT


def _compositions(k):
    """Every split of classes 1..k into contiguous ranges, as lists of (i, j)."""
    for cuts in itertools.product((0, 1), repeat=k - 1):
        parts, i = [], 1
        for c, cut in enumerate(cuts, start=1):
            if cut:
                parts.append((i, c))
                i = c + 1
        parts.append((i, k))
        yield parts


@pytest.mark.parametrize("seed", range(6))
def test_best_partition_matches_brute_force(seed):
    import numpy as np
    rng = np.random.default_rng(seed)
    cost = {}
    for i in range(1, A.CLASSES + 1):
        for j in range(i, A.CLASSES + 1):
            # launch tail + work growing with the range: neither extreme always wins
            ms = float(rng.uniform(0.05, 0.4) + sum(rng.uniform(0.1, 1.0) * k * k for k in range(i, j + 1)) / 20)
            cost[(i, j)] = (ms, int(rng.choice([64, 128, 256, 512, 1024])))
    total, parts = A.best_partition(cost)
    brute = min(sum(cost[p][0] for p in comp) for comp in _compositions(A.CLASSES))
    assert total == pytest.approx(brute)
    assert sum(ms for _, _, ms in parts) == pytest.approx(total)
    edges = [e for e, _, _ in parts]
    assert edges == sorted(edges) and edges[-1] == 32 * A.CLASSES
    for e, team, ms in parts:
        assert e % 32 == 0


def test_best_partition_skips_empty_classes():
    """Classes 1 and 2 hold no circuits (their ranges cost nothing); every
    launch costs 0.5 ms plus 1 ms per non-empty class: one launch is best."""
    cost = {}
    for i in range(1, A.CLASSES + 1):
        for j in range(i, A.CLASSES + 1):
            cost[(i, j)] = None if j <= 2 else (0.5 + (j - max(i, 3) + 1), 256)
    total, parts = A.best_partition(cost)
    assert total == pytest.approx(6.5)
    assert len(parts) == 1 and parts[0][0] == 256


def test_word_class():
    assert [A.word_class(n) for n in (1, 32, 33, 64, 65, 255, 256)] == [1, 1, 2, 2, 3, 8, 8]


def test_committed_tuning_table_is_valid():
    teams = BT.load_tuning()
    assert list(teams) == sorted(teams) and max(teams) == 256
    from paper_2408_00384_amd import _binding as B
    assert all(t in B.BATCH_TEAMS for t in teams.values())
    rec = json.load(open(BT.TUNING_PATH))
    assert rec["best_total_ms"] <= rec["fixed_buckets_ms"] * 1.02


def test_check_teams_rejects_bad_tables():
    with pytest.raises(ValueError):
        BT.check_teams({256: 96})
    with pytest.raises(ValueError):
        BT.check_teams({300: 256})
    assert list(BT.check_teams({256: 256, 64: 128})) == [64, 256]


def _layer_ops(n, depth, seed):
    from inputs import layered_circuit
    from paper_2408_00384_amd import _binding as B
    c = layered_circuit(n, depth, 1, gen_seed=seed, circuit_id=0)
    return B.cliff_encode_layers(c.n, c.h, c.s, c.ctrl, c.tgt)


def _excess(stream, offs, n):
    """Mean over the kernel's access groups (and halves, W >= 5) of the
    largest number of ops sharing a bank class, minus one: the extra LDS
    cycles of a group's column accesses, first and second qubits apart."""
    import numpy as np
    W = (2 * n + 63) // 64
    wq = 4 if W >= 5 else (1 if W <= 1 else 1 << (W - 1).bit_length())
    P = 4 if W >= 5 else 32 // wq
    group = 8 if W >= 5 else P
    mask = np.uint64((1 << 24) - 1)
    tot, cnt = 0, 0
    for l in range(len(offs) - 1):
        L = stream[offs[l]:offs[l + 1]]
        for g0 in range(0, len(L), group):
            g = L[g0:g0 + group]
            for h in ((g[0::2], g[1::2]) if W >= 5 else (g,)):
                if len(h) == 0:
                    continue
                two = (h >> np.uint64(62)) != 0
                for q in ((h & mask).astype(np.int64) % P,
                          ((h >> np.uint64(24)) & mask).astype(np.int64)[two] % P):
                    if len(q):
                        tot += np.bincount(q).max() - 1
                        cnt += 1
    return tot / max(cnt, 1)


@pytest.mark.parametrize("n", [1, 20, 32, 33, 64, 65, 100, 128, 129, 160, 200, 255, 256])
def test_batch_order_is_a_permutation_per_layer_and_spreads_banks(n):
    """Each layer keeps its ops (as a multiset) and only they move; the order
    is deterministic; and the ops the kernel issues together share bank
    classes (first qubits, and second qubits of two-qubit ops, mod 32 / Wq;
    mod 4 per slot parity when W >= 5) far less than in the encoder's order."""
    import numpy as np
    from paper_2408_00384_amd import _binding as B
    ops, offs = _layer_ops(n, 12, [n, 7])
    got = B.cliff_batch_order_ops(n, ops.copy(), offs)
    again = B.cliff_batch_order_ops(n, ops.copy(), offs)
    assert np.array_equal(got, again)
    for l in range(len(offs) - 1):
        a, b = ops[offs[l]:offs[l + 1]], got[offs[l]:offs[l + 1]]
        assert sorted(a.tolist()) == sorted(b.tolist())
    before, after = _excess(ops, offs, n), _excess(got, offs, n)
    W = (2 * n + 63) // 64
    if W >= 5:     # groups of 2 x 4 ops over 4 classes
        assert after <= 0.3 * before + 1e-9 and after < 0.35, (before, after)
    elif W >= 3:   # 8 ops over 8 classes
        assert after <= 0.5 * before + 1e-9 and after < 0.7, (before, after)
    else:          # 16 or 32 ops over as many classes: no worse
        assert after <= before + 1e-9, (before, after)


def test_batch_order_rejects_bad_arguments():
    import numpy as np
    from paper_2408_00384_amd import _binding as B
    ops, offs = _layer_ops(40, 3, 1)
    for n in (0, 257):
        with pytest.raises(B.CliffError):
            B.cliff_batch_order_ops(n, ops.copy(), offs)
    bad = offs.copy()
    bad[1], bad[2] = bad[2], bad[1]
    if bad[1] > bad[2]:
        with pytest.raises(B.CliffError):
            B.cliff_batch_order_ops(40, ops.copy(), bad)
    with pytest.raises(ValueError):
        B.cliff_batch_order_ops(40, ops.astype(np.int64), offs)

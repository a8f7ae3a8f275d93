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

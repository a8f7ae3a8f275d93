"""Batched persistent kernel vs the CPU oracle (bit-exact outcome bytes)."""
import numpy as np
import pytest
import torch

import oracle
from inputs import batch_circuit, layered_circuit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2408_00384_amd import Context
    stream = torch.cuda.Stream()
    c = Context(0, stream)
    yield c
    c.close()


def _mixed_circuits(count=36, seed=7):
    rng = np.random.default_rng(seed)
    ns = list(rng.integers(1, 257, size=count - 8)) + [1, 2, 31, 32, 33, 64, 65, 256]
    out = []
    for i, n in enumerate(ns):
        n = int(n)
        depth = int(rng.integers(0, 12))
        shots = int(rng.choice([1, 3, 4, 17, 64]))
        out.append(layered_circuit(n, depth, shots, gen_seed=[seed, i], circuit_id=1000 + i))
    return out


def _check(circs, outs):
    for c, o in zip(circs, outs):
        for s in range(c.shots):
            ref, _ = oracle.run_shot(c, s)
            assert np.array_equal(o[s], ref), "circuit %d (n=%d) shot %d" % (c.circuit_id, c.n, s)


def test_batch_matches_oracle_default_teams(ctx):
    from paper_2408_00384_amd.batch import BatchPlan
    circs = _mixed_circuits()
    with torch.cuda.stream(ctx.stream):
        plan = BatchPlan(ctx, circs).run()
        outs = plan.outcomes()
    assert plan.status() == dict(rejected=0, anomalies=0)
    _check(circs, outs)


TEAMS = (64, 128, 256, 512, 1024)


@pytest.mark.parametrize("team", TEAMS)
@pytest.mark.parametrize("maxn", (64, 128, 256))
def test_every_team_config_is_bit_identical(ctx, team, maxn):
    from paper_2408_00384_amd.batch import BatchPlan
    rng = np.random.default_rng(maxn)
    lo = {64: 1, 128: 65, 256: 129}[maxn]
    circs = [layered_circuit(int(n), int(rng.integers(1, 8)), 4, gen_seed=[3, maxn, i], circuit_id=i)
             for i, n in enumerate(rng.integers(lo, maxn + 1, size=6))]
    with torch.cuda.stream(ctx.stream):
        plan = BatchPlan(ctx, circs, teams={maxn: team}).run()
        outs = plan.outcomes()
    assert plan.status() == dict(rejected=0, anomalies=0)
    _check(circs, outs)


def test_batched_workload_sample_and_graph_replay(ctx):
    """Circuits of the 4,096-circuit workload (n in [8, 256], depth in [n, 4n],
    4 shots): a sample checked against the oracle, replayed from a HIP graph."""
    from inputs import batch_sizes
    from paper_2408_00384_amd.batch import BatchPlan
    ns, depths = batch_sizes()
    idx = [0, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144]
    circs = [batch_circuit(i, ns, depths) for i in idx]
    with torch.cuda.stream(ctx.stream):
        plan = BatchPlan(ctx, circs).capture()
        outs = []
        for rep in range(3):
            plan.d_out.zero_()
            torch.cuda.current_stream().synchronize()
            plan.run()
            outs.append(plan.outcomes())
    for rep in (1, 2):
        assert all(np.array_equal(a, b) for a, b in zip(outs[0], outs[rep]))
    assert plan.status() == dict(rejected=0, anomalies=0)
    _check(circs, outs[0])
    plan.close()


def test_rejects_oversized_descriptors(ctx):
    from paper_2408_00384_amd import _binding as B
    from paper_2408_00384_amd.batch import BatchPlan
    circs = [layered_circuit(100, 2, 2, gen_seed=1, circuit_id=0),
             layered_circuit(20, 2, 2, gen_seed=2, circuit_id=1)]
    with torch.cuda.stream(ctx.stream):
        plan = BatchPlan(ctx, circs)
        order = torch.tensor([0, 1], dtype=torch.int32, device="cuda:0")
        torch.cuda.synchronize()
        B.cliff_batch_run(ctx.handle, plan.d_descs.data_ptr(), plan.d_ops.data_ptr(),
                          plan.d_offs.data_ptr(), plan.d_out.data_ptr(), order.data_ptr(), 2,
                          plan.seed, plan.d_work.data_ptr(), 64, 64, 2)
        st = B.cliff_batch_status(ctx.handle, plan.d_work.data_ptr())
    assert st["rejected"] == 1
    out = plan.d_out.cpu().numpy()
    d = plan.descs[1]
    got = out[int(d["out_off"]): int(d["out_off"]) + 2 * 20].reshape(2, 20)
    for s in range(2):
        assert np.array_equal(got[s], oracle.run_shot(circs[1], s)[0])


def _det_heavy_circuits(maxn, seed, count=6):
    """Circuits whose measure-all is mostly deterministic after its first
    random outcome, so the outcomes depend on the batch kernel's sign
    arithmetic and not only on the Philox bits: half shallow (one layer, H on
    about a quarter of the qubits, so many CNOT pairs form Bell pairs), half
    GHZ-like (H on qubit 0 only, then CNOT layers: the state is |0...0> +
    |v>, whose first measured qubit in supp(v) is random and every other
    outcome follows from it)."""
    rng = np.random.default_rng([seed, maxn])
    lo = {64: 1, 128: 65, 256: 129}[maxn]
    out = []
    for i in range(count):
        n = int(rng.integers(max(lo, 4), maxn + 1))
        shots = int(rng.choice([1, 17, 64]))
        if i % 2 == 0:
            c = layered_circuit(n, 1, shots, gen_seed=[seed, maxn, i], circuit_id=2000 + i)
            c.h[:] = (rng.random((1, n)) < 0.25).astype(np.uint8)
        else:
            c = layered_circuit(n, 6, shots, gen_seed=[seed, maxn, i], circuit_id=2000 + i)
            c.h[:] = 0
            c.s[:] = 0
            c.h[0, 0] = 1
        out.append(c)
    return out


@pytest.mark.parametrize("team", TEAMS)
@pytest.mark.parametrize("maxn", (64, 128, 256))
def test_mostly_deterministic_circuits_every_team_config(ctx, team, maxn):
    """Every kernel instance against the oracle, every shot, on circuits
    where at least 30 % of the outcomes after the first random one are
    deterministic (each then depends on the signs the kernel tracked)."""
    from paper_2408_00384_amd.batch import BatchPlan
    circs = _det_heavy_circuits(maxn, seed=team)
    with torch.cuda.stream(ctx.stream):
        plan = BatchPlan(ctx, circs, teams={maxn: team}).run()
        outs = plan.outcomes()
    assert plan.status() == dict(rejected=0, anomalies=0)
    det = after = 0
    for c, o in zip(circs, outs):
        for s in range(c.shots):
            ref, kinds = oracle.run_shot(c, s)
            assert np.array_equal(o[s], ref), "circuit %d (n=%d) shot %d" % (c.circuit_id, c.n, s)
        first = int(np.argmax(kinds)) if kinds.any() else len(kinds)
        det += int((kinds[first + 1:] == 0).sum())
        after += max(0, len(kinds) - first - 1)
    assert after > 0 and det >= 0.3 * after, (det, after)


def test_rejects_shots_above_the_launch_bound(ctx):
    """LDS holds max_shots sign columns: a circuit with more shots is skipped
    and counted, the others run (outcomes against the oracle)."""
    from paper_2408_00384_amd import _binding as B
    from paper_2408_00384_amd.batch import BatchPlan
    circs = [layered_circuit(40, 3, 5, gen_seed=4, circuit_id=0),
             layered_circuit(40, 3, 3, gen_seed=5, circuit_id=1)]
    with torch.cuda.stream(ctx.stream):
        plan = BatchPlan(ctx, circs)
        order = torch.tensor([0, 1], dtype=torch.int32, device="cuda:0")
        torch.cuda.synchronize()
        B.cliff_batch_run(ctx.handle, plan.d_descs.data_ptr(), plan.d_ops.data_ptr(),
                          plan.d_offs.data_ptr(), plan.d_out.data_ptr(), order.data_ptr(), 2,
                          plan.seed, plan.d_work.data_ptr(), 128, 40, 4)
        st = B.cliff_batch_status(ctx.handle, plan.d_work.data_ptr())
    assert st == dict(rejected=1, anomalies=0)
    out = plan.d_out.cpu().numpy()
    d = plan.descs[1]
    got = out[int(d["out_off"]): int(d["out_off"]) + 3 * 40].reshape(3, 40)
    for s_ in range(3):
        assert np.array_equal(got[s_], oracle.run_shot(circs[1], s_)[0])


@pytest.mark.parametrize("team,maxn,shots", [(96, 64, 4), (2048, 64, 4), (64, 0, 4), (64, 257, 4),
                                             (64, 64, 0), (64, 64, 65)])
def test_launch_bounds_out_of_range(ctx, team, maxn, shots):
    from paper_2408_00384_amd import _binding as B
    from paper_2408_00384_amd.batch import BatchPlan
    circs = [layered_circuit(10, 2, 2, gen_seed=1, circuit_id=0)]
    with torch.cuda.stream(ctx.stream):
        plan = BatchPlan(ctx, circs)
        order = torch.tensor([0], dtype=torch.int32, device="cuda:0")
        torch.cuda.synchronize()
        with pytest.raises(B.CliffError):
            B.cliff_batch_run(ctx.handle, plan.d_descs.data_ptr(), plan.d_ops.data_ptr(),
                              plan.d_offs.data_ptr(), plan.d_out.data_ptr(), order.data_ptr(), 1,
                              plan.seed, plan.d_work.data_ptr(), team, maxn, shots)


def test_tuned_choices_are_bit_identical(ctx):
    """The autotuner's table (bucket edges and a team per bucket) against the
    fixed 64 / 128 / 256 buckets with their default teams and against one
    bucket of every circuit: identical outcome bytes on circuits of the
    batched workload spread over every row-word class, and the oracle on a
    sample of them (every shot)."""
    from inputs import batch_circuit, batch_sizes
    from paper_2408_00384_amd.batch import DEFAULT_TEAMS, BatchPlan, load_tuning
    tuned = load_tuning()
    assert max(tuned) == 256
    ns, depths = batch_sizes()
    order = np.argsort(ns, kind="stable")
    idx = [int(order[k]) for k in np.linspace(0, len(order) - 1, 48).astype(int)]
    circs = [batch_circuit(i, ns, depths) for i in idx]
    outs = {}
    for name, teams in (("tuned", tuned), ("fixed", DEFAULT_TEAMS), ("one", {256: 256})):
        with torch.cuda.stream(ctx.stream):
            plan = BatchPlan(ctx, circs, teams=teams).run()
            outs[name] = plan.outcomes()
        assert plan.status() == dict(rejected=0, anomalies=0), name
    for name in ("fixed", "one"):
        assert all(np.array_equal(a, b) for a, b in zip(outs["tuned"], outs[name])), name
    _check(circs[::6], outs["tuned"][::6])

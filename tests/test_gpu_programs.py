"""GPU parity for circuits with mid-circuit measurement, reset and classically
conditioned Paulis (all shots on one tableau, outcomes in a device record),
against the oracle run shot by shot: every recorded outcome, the random
flags and each shot's final tableau bit for bit."""
import numpy as np
import pytest

import oracle
from inputs import random_program
from inputs.programs import Program

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2408_00384_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(params=["step", "persistent"])
def measure_mode(request, ctx):
    from paper_2408_00384_amd import (MEASURE_AUTO, MEASURE_PERSISTENT, MEASURE_STEP,
                                      cliff_ctx_set_measure_mode)
    cliff_ctx_set_measure_mode(ctx.handle, MEASURE_STEP if request.param == "step" else MEASURE_PERSISTENT)
    yield request.param
    cliff_ctx_set_measure_mode(ctx.handle, MEASURE_AUTO)


@pytest.mark.parametrize("n", [1, 3, 5, 33, 100, 300, 2100])
def test_programs_match_oracle(ctx, measure_mode, n):
    from paper_2408_00384_amd.program import run_program
    prog = random_program(n, 10, 4, [31, n], circuit_id=n)
    rec, rnd, tab = run_program(ctx, prog)
    gx, gz, gr = tab.export()
    for s in range(prog.shots):
        want, kinds, t = oracle.run_program(prog, s)
        assert np.array_equal(rec[s], want), "record differs (shot %d)" % s
        assert np.array_equal(rnd, kinds), "random flags differ"
        x, z, r = t.get()
        assert np.array_equal(gx, x) and np.array_equal(gz, z), "x/z differ"
        assert np.array_equal(gr[s], r), "signs differ (shot %d)" % s
    assert tab.anomalies() == 0


def test_teleportation_on_device(ctx):
    """Teleport the six single-qubit stabilizer states, 16 shots each: after
    the record-conditioned corrections qubit 2 measures deterministically in
    the prepared state's basis, in every shot."""
    from inputs import OP_CNOT, OP_H, OP_S, OP_SDG, OP_X
    from paper_2408_00384_amd import BASIS_X, BASIS_Y, BASIS_Z
    from paper_2408_00384_amd.program import run_program
    preps = [([], BASIS_Z, 0), ([OP_X], BASIS_Z, 1), ([OP_H], BASIS_X, 0), ([OP_X, OP_H], BASIS_X, 1),
             ([OP_H, OP_S], BASIS_Y, 0), ([OP_H, OP_SDG], BASIS_Y, 1)]
    for ops, basis, want in preps:
        steps = [("gates", np.array(ops + [OP_H, OP_CNOT, OP_CNOT, OP_H], np.uint8),
                  np.array([0] * len(ops) + [1, 1, 0, 0], np.uint32),
                  np.array([0] * len(ops) + [0, 2, 1, 0], np.uint32)),
                 ("measure", np.array([0, 1], np.uint32)),
                 ("cond", np.array([2, 2], np.uint32), np.array([1, 3], np.uint8), np.array([1, 0], np.uint32))]
        rec, rnd, tab = run_program(ctx, Program(n=3, steps=steps, shots=16))
        assert rnd.tolist() == [1, 1]
        assert len({tuple(r) for r in rec.tolist()}) > 1
        out, kinds = tab.measure_bases([2], [basis], m0=5)
        assert kinds.tolist() == [0] and set(out[:, 0].tolist()) == {want}


def test_reset_ghz_all_shots(ctx):
    from inputs import OP_CNOT, OP_H
    from paper_2408_00384_amd.program import run_program
    n = 10
    ops = np.array([OP_H] + [OP_CNOT] * (n - 1), np.uint8)
    a = np.array([0] + list(range(n - 1)), np.uint32)
    b = np.array([0] + list(range(1, n)), np.uint32)
    prog = Program(n=n, steps=[("gates", ops, a, b), ("reset", np.arange(n, dtype=np.uint32))], shots=64)
    rec, rnd, tab = run_program(ctx, prog)
    assert rnd[0] == 1 and rnd[1:].sum() == 0
    assert all(len(set(r)) == 1 for r in rec.tolist())        # GHZ: one value per shot
    assert len({r[0] for r in rec.tolist()}) == 2
    out, kinds = tab.measure(np.arange(n), m0=n)
    assert out.sum() == 0 and kinds.sum() == 0


def test_outcome_counts_bell(ctx):
    from inputs import OP_CNOT, OP_H
    from paper_2408_00384_amd.program import outcome_counts, run_program
    prog = Program(n=2, steps=[("gates", np.array([OP_H, OP_CNOT], np.uint8), np.array([0, 0], np.uint32),
                                np.array([0, 1], np.uint32)), ("measure", np.array([0, 1], np.uint32))],
                   shots=1000)
    rec, _, _ = run_program(ctx, prog)
    counts = outcome_counts(rec)
    assert set(counts) == {"00", "11"} and sum(counts.values()) == 1000
    want = [oracle.random_bit(prog.seed, 0, s, 0) for s in range(1000)]
    assert counts["11"] == sum(want)


def test_conditional_pauli_errors(ctx):
    import torch
    from paper_2408_00384_amd import CLIFF_EINVAL, CliffError, DeviceTableau, cliff_apply_cond_paulis
    t = DeviceTableau(ctx, 4, 2)
    rec = torch.zeros((2, 3), dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    for q, p, c in [([4], [1], [0]), ([0], [0], [0]), ([0], [4], [0]), ([0], [1], [3])]:
        with pytest.raises(CliffError) as e:
            cliff_apply_cond_paulis(t.handle, q, p, c, rec.data_ptr(), 3)
        assert e.value.code == CLIFF_EINVAL


@pytest.mark.parametrize("n", [3, 33, 200])
def test_conditioned_gate_programs_match_oracle(ctx, n):
    """Gate lists conditioned on recorded outcomes: every shot on a tableau of
    its own; outcomes, random flags and each shot's tableau against the
    oracle."""
    from paper_2408_00384_amd.program import run_program
    prog = random_program(n, 12, 5, [33, n], circuit_id=n, conditioned_gates=True)
    assert any(st[0] == "cgates" for st in prog.steps)
    rec, rnd, tabs = run_program(ctx, prog)
    for s in range(prog.shots):
        want, kinds, t = oracle.run_program(prog, s)
        assert np.array_equal(rec[s], want), "record differs (shot %d)" % s
        assert np.array_equal(rnd[s], kinds), "random flags differ (shot %d)" % s
        gx, gz, gr = tabs[s].export()
        x, z, r = t.get()
        assert np.array_equal(gx, x) and np.array_equal(gz, z) and np.array_equal(gr[0], r)


def test_per_shot_mode_equals_shared_mode(ctx):
    """The per-shot runner on a program without conditioned gates gives the
    shared-tableau runner's outcomes and tableaux."""
    from paper_2408_00384_amd.program import _run_per_shot, run_program
    prog = random_program(40, 8, 4, [34], circuit_id=2)
    rec, rnd, tab = run_program(ctx, prog)
    rec2, rnd2, tabs = _run_per_shot(ctx, prog)
    assert np.array_equal(rec, rec2) and all(np.array_equal(rnd, r) for r in rnd2)
    gx, gz, gr = tab.export()
    for s, t in enumerate(tabs):
        x, z, r = t.export()
        assert np.array_equal(gx, x) and np.array_equal(gz, z) and np.array_equal(gr[s], r[0])

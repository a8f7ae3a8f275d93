"""Failure handling of the register-resident measurement path, forced from the
host: the context's injection makes every workgroup give up at a chosen
measurement, as it would after a timed-out wait, so every kernel still exits
normally.  The error must surface at the next synchronizing call, the chunks
after the aborted one must do nothing, the flag must be lowered by the report,
and the tableau must be usable again once re-initialized."""
import numpy as np
import pytest

from inputs import layered_circuit, random_gate_list

pytestmark = pytest.mark.gpu

NONE = 2**64 - 1


@pytest.fixture(scope="module")
def ctx():
    from paper_2408_00384_amd import Context
    c = Context(0)
    yield c
    c.close()


def _mode(ctx, mode):
    from paper_2408_00384_amd import cliff_ctx_set_measure_mode
    cliff_ctx_set_measure_mode(ctx.handle, mode)


@pytest.fixture
def persistent(ctx):
    from paper_2408_00384_amd import MEASURE_AUTO, MEASURE_PERSISTENT, cliff_ctx_inject_abort
    _mode(ctx, MEASURE_PERSISTENT)
    yield
    cliff_ctx_inject_abort(ctx.handle, NONE)
    _mode(ctx, MEASURE_AUTO)


def _step_reference(ctx, c):
    from paper_2408_00384_amd import MEASURE_PERSISTENT, MEASURE_STEP, DeviceTableau
    _mode(ctx, MEASURE_STEP)
    t = DeviceTableau(ctx, c.n, c.shots).apply_circuit_gates(c)
    out, kinds = t.measure(c.qubits, seed=c.seed, circuit=c.circuit_id)
    tab = t.export()
    _mode(ctx, MEASURE_PERSISTENT)
    return out, kinds, tab


@pytest.mark.parametrize("at", [0, 300, 2047])
def test_abort_surfaces_and_later_chunks_skip(ctx, persistent, at):
    """n = 2,048 measured in 8 chunks of 256: abort in the first, a middle
    and the last chunk.  Only the chunks before the aborted one count their
    measurements."""
    from paper_2408_00384_amd import (CLIFF_EINTERNAL, CliffError, DeviceTableau, cliff_ctx_inject_abort,
                                      cliff_tab_counters, cliff_tab_reset_counters)
    c = layered_circuit(2048, 4, 4, gen_seed=[41], circuit_id=3)
    want_out, want_kinds, want_tab = _step_reference(ctx, c)
    t = DeviceTableau(ctx, c.n, c.shots).apply_circuit_gates(c)
    cliff_tab_reset_counters(t.handle)
    cliff_ctx_inject_abort(ctx.handle, at)
    with pytest.raises(CliffError) as e:
        t.measure(c.qubits, seed=c.seed, circuit=c.circuit_id)
    assert e.value.code == CLIFF_EINTERNAL
    cnt = cliff_tab_counters(t.handle)          # the report lowered the flag
    assert cnt["random"] + cnt["deterministic"] == (at // 256) * 256
    # the same tableau, re-initialized, gives the step path's results
    t.init_zero().apply_circuit_gates(c)
    out, kinds = t.measure(c.qubits, seed=c.seed, circuit=c.circuit_id)
    assert np.array_equal(out, want_out) and np.array_equal(kinds, want_kinds)
    for a, b in zip(t.export(), want_tab):
        assert np.array_equal(a, b)


def test_abort_in_record_path_surfaces_at_readout(ctx, persistent):
    """Outcomes into a device record raise nothing at the call; the next
    synchronizing call reports the abort once."""
    import torch
    from paper_2408_00384_amd import (CLIFF_EINTERNAL, CliffError, DeviceTableau, cliff_ctx_inject_abort,
                                      cliff_measure_record)
    n = 300
    rng = np.random.Generator(np.random.PCG64(42))
    ops, a, b = random_gate_list(rng, n, 4 * n, full=True)
    t = DeviceTableau(ctx, n, 3).apply_gates(ops, a, b)
    rec = torch.zeros((3, 8), dtype=torch.uint8, device="cuda:0")
    torch.cuda.synchronize()
    cliff_ctx_inject_abort(ctx.handle, 2)
    cliff_measure_record(t.handle, np.arange(8, dtype=np.uint32), rec.data_ptr(), 8, 0)
    with pytest.raises(CliffError) as e:
        t.anomalies()
    assert e.value.code == CLIFF_EINTERNAL
    assert t.anomalies() == 0


def test_injection_counts_down_over_calls(ctx, persistent):
    """An injection at measurement 5 passes a first call of 4 measurements and
    stops the second call at its second measurement; once spent, it stops
    nothing."""
    from paper_2408_00384_amd import CLIFF_EINTERNAL, CliffError, DeviceTableau, cliff_ctx_inject_abort
    c = layered_circuit(200, 6, 2, gen_seed=[43])
    want_out, want_kinds, _ = _step_reference(ctx, c)
    t = DeviceTableau(ctx, c.n, c.shots).apply_circuit_gates(c)
    cliff_ctx_inject_abort(ctx.handle, 5)
    out, kinds = t.measure(c.qubits[:4], seed=c.seed, circuit=c.circuit_id)
    assert np.array_equal(out, want_out[:, :4]) and np.array_equal(kinds, want_kinds[:4])
    with pytest.raises(CliffError) as e:
        t.measure(c.qubits[4:8], seed=c.seed, circuit=c.circuit_id, m0=4)
    assert e.value.code == CLIFF_EINTERNAL
    t.init_zero().apply_circuit_gates(c)
    out, kinds = t.measure(c.qubits, seed=c.seed, circuit=c.circuit_id)
    assert np.array_equal(out, want_out) and np.array_equal(kinds, want_kinds)


def test_injection_on_step_path_is_inert(ctx, persistent):
    """A measurement that runs on the step path cannot abort; it spends the
    injection all the same."""
    from paper_2408_00384_amd import MEASURE_STEP, DeviceTableau, cliff_ctx_inject_abort
    c = layered_circuit(100, 5, 2, gen_seed=[44])
    want_out, want_kinds, _ = _step_reference(ctx, c)
    t = DeviceTableau(ctx, c.n, c.shots).apply_circuit_gates(c)
    cliff_ctx_inject_abort(ctx.handle, 0)
    _mode(ctx, MEASURE_STEP)
    out, _ = t.measure(c.qubits[:1], seed=c.seed, circuit=c.circuit_id)
    from paper_2408_00384_amd import MEASURE_PERSISTENT
    _mode(ctx, MEASURE_PERSISTENT)
    out2, _ = t.measure(c.qubits[1:], seed=c.seed, circuit=c.circuit_id, m0=1)
    assert np.array_equal(np.concatenate([out, out2], axis=1), want_out)

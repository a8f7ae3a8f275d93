"""The blocked pass of the register-resident measurement (runs of random
measurements applied as one low-rank update per block of up to 32) against
the CPU oracle and against the per-measurement kernels, bit for bit: tableau
bits, every shot's signs, outcomes and the random/deterministic flags.

The broader suites run it too: tests/test_gpu_parity.py's measurement tests
take MEASURE_BLOCKED as a third mode, and the automatic mode uses it from
n = 2,048 on (the stored n = 10,000 oracle digests)."""
import numpy as np
import pytest

import oracle
from inputs import layered_circuit

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
def blocked(ctx):
    from paper_2408_00384_amd import MEASURE_AUTO, MEASURE_BLOCKED
    _mode(ctx, MEASURE_BLOCKED)
    yield
    _mode(ctx, MEASURE_AUTO)


def _oracle_run(c, q, shots):
    ref = oracle.Tableau(c.n).apply_circuit_gates(c)
    outs, kinds, tabs = [], None, []
    for s in range(shots):
        r = ref.clone()
        o, k = r.measure_list(q, seed=c.seed, circuit=c.circuit_id, shot=s)
        outs.append(o)
        kinds = k
        tabs.append(r.get())
    return np.stack(outs), kinds, tabs


def _check(ctx, c, q, shots):
    from paper_2408_00384_amd import DeviceTableau
    t = DeviceTableau(ctx, c.n, shots).apply_circuit_gates(c)
    out, rnd = t.measure(q, seed=c.seed, circuit=c.circuit_id)
    gx, gz, gr = t.export()
    want_out, want_kinds, tabs = _oracle_run(c, q, shots)
    assert np.array_equal(rnd, want_kinds)
    assert np.array_equal(out, want_out)
    for s, (x, z, r) in enumerate(tabs):
        assert np.array_equal(gx, x), "x bits"
        assert np.array_equal(gz, z), "z bits"
        assert np.array_equal(gr[s], r), "signs of shot %d" % s
    assert t.anomalies() == 0
    t.close()
    return rnd


@pytest.mark.parametrize("n,depth", [(64, 12), (65, 12), (300, 12), (1000, 16), (1000, 40)])
def test_dense_measure_all_vs_oracle(ctx, blocked, n, depth):
    """Deep circuits: nearly every outcome random, so whole blocks of 32 run
    through the low-rank update (n = 1,000: chunks of 128, four blocks each)."""
    c = layered_circuit(n, depth, 3, gen_seed=[60, n, depth], circuit_id=11)
    rnd = _check(ctx, c, c.qubits, 3)
    assert rnd.mean() > 0.9


@pytest.mark.parametrize("n,depth", [(200, 1), (600, 1), (600, 2), (999, 3)])
def test_shallow_mixed_vs_oracle(ctx, blocked, n, depth):
    """Shallow circuits mix random and deterministic outcomes: each chunk's
    blocked pass stops at its first deterministic measurement and the
    per-measurement kernels finish the chunk from the count it left."""
    c = layered_circuit(n, depth, 2, gen_seed=[61, n, depth], circuit_id=12)
    rnd = _check(ctx, c, c.qubits, 2)
    assert 0.05 < rnd.mean() < 0.95


def test_repeats_and_partial_lists_vs_oracle(ctx, blocked):
    """A repeated qubit inside a block (deterministic re-measurement), a list
    not a multiple of 32 long, and a second call continuing the first."""
    from paper_2408_00384_amd import DeviceTableau
    n, shots = 700, 3
    c = layered_circuit(n, 14, shots, gen_seed=[62], circuit_id=13)
    q1 = np.concatenate([np.arange(0, 40), [5, 39], np.arange(600, 650)]).astype(np.uint32)
    q2 = np.arange(40, 93).astype(np.uint32)
    t = DeviceTableau(ctx, n, shots).apply_circuit_gates(c)
    o1, k1 = t.measure(q1, seed=c.seed, circuit=13)
    o2, k2 = t.measure(q2, seed=c.seed, circuit=13, m0=len(q1))
    gx, gz, gr = t.export()
    ref = oracle.Tableau(n).apply_circuit_gates(c)
    q = np.concatenate([q1, q2])
    for s in range(shots):
        r = ref.clone()
        o, k = r.measure_list(q, seed=c.seed, circuit=13, shot=s)
        assert np.array_equal(np.concatenate([o1[s], o2[s]]), o)
        assert np.array_equal(np.concatenate([k1, k2]), k)
        x, z, rr = r.get()
        assert np.array_equal(gx, x) and np.array_equal(gz, z) and np.array_equal(gr[s], rr)
    assert k1[40] == 0 and k1[41] == 0     # the repeats are deterministic
    t.close()


@pytest.mark.parametrize("n,shots", [(2100, 3), (6000, 2), (7000, 2), (10000, 1)])
def test_large_prefix_vs_oracle(ctx, blocked, n, shots):
    """Register-resident sizes with 2..5 row words per lane: a 70-measurement
    prefix of measure-all (three blocks, the last partial) against the
    oracle, full tableau compared."""
    c = layered_circuit(n, 14, shots, gen_seed=[63, n], circuit_id=14)
    q = np.arange(70, dtype=np.uint32)
    rnd = _check(ctx, c, q, shots)
    assert rnd.all()


def test_counters_match_per_measurement_path(ctx):
    """Random and deterministic counts and the pivot-row support the device
    counters accumulate are those of the per-measurement kernels."""
    from paper_2408_00384_amd import (MEASURE_AUTO, MEASURE_BLOCKED, MEASURE_PERSISTENT, DeviceTableau,
                                      cliff_tab_counters, cliff_tab_reset_counters)
    res = {}
    for n, depth in ((1000, 16), (600, 2)):
        c = layered_circuit(n, depth, 2, gen_seed=[64, n], circuit_id=15)
        for mode in (MEASURE_PERSISTENT, MEASURE_BLOCKED):
            _mode(ctx, mode)
            t = DeviceTableau(ctx, n, 2).apply_circuit_gates(c)
            cliff_tab_reset_counters(t.handle)
            t.measure(c.qubits, seed=c.seed, circuit=15)
            res[(n, mode)] = cliff_tab_counters(t.handle)
            t.close()
        assert res[(n, MEASURE_PERSISTENT)] == res[(n, MEASURE_BLOCKED)]
    _mode(ctx, MEASURE_AUTO)


@pytest.mark.parametrize("at", [0, 100, 700, 1499])
def test_abort_in_blocked_pass(ctx, at):
    """The injected abort stops the blocked pass like a timed-out wait: the
    call reports CLIFF_EINTERNAL, and the tableau, re-initialized, gives the
    oracle's results.  The device counters hold the chunks before the aborted
    one (n = 1,500: chunks of 256) and, within it, at most the measurements
    before `at` (the blocked pass may have completed a prefix of the chunk
    and stopped at a deterministic measurement before the per-measurement
    kernel reached `at`)."""
    from paper_2408_00384_amd import (CLIFF_EINTERNAL, MEASURE_AUTO, MEASURE_BLOCKED, CliffError, DeviceTableau,
                                      cliff_ctx_inject_abort, cliff_tab_counters, cliff_tab_reset_counters)
    n = 1500
    c = layered_circuit(n, 12, 2, gen_seed=[65], circuit_id=16)
    _mode(ctx, MEASURE_BLOCKED)
    try:
        t = DeviceTableau(ctx, n, 2).apply_circuit_gates(c)
        cliff_tab_reset_counters(t.handle)
        cliff_ctx_inject_abort(ctx.handle, at)
        with pytest.raises(CliffError) as e:
            t.measure(c.qubits, seed=c.seed, circuit=16)
        assert e.value.code == CLIFF_EINTERNAL
        cnt = cliff_tab_counters(t.handle)
        assert (at // 256) * 256 <= cnt["random"] + cnt["deterministic"] <= at
        t.init_zero().apply_circuit_gates(c)
        out, kinds = t.measure(c.qubits[:64], seed=c.seed, circuit=16)
        ref = oracle.Tableau(n).apply_circuit_gates(c)
        for s in range(2):
            o, k = ref.clone().measure_list(c.qubits[:64], seed=c.seed, circuit=16, shot=s)
            assert np.array_equal(out[s], o) and np.array_equal(kinds, k)
        t.close()
    finally:
        cliff_ctx_inject_abort(ctx.handle, NONE)
        _mode(ctx, MEASURE_AUTO)


@pytest.mark.parametrize("n,depth", [(8500, 1), (10000, 2)])
def test_large_mixed_equals_step(ctx, n, depth):
    """Above n = 8192 (five planner word groups; chunks of 2048, the pass
    ending with a short one) on a shallow circuit that mixes random and
    deterministic outcomes: each chunk's blocked pass stops at its first
    deterministic measurement and the per-measurement kernels finish the
    chunk from the count it left.  Tableau, outcomes and both shots' signs
    equal the step path's (itself checked against the oracle elsewhere)."""
    from paper_2408_00384_amd import MEASURE_BLOCKED, MEASURE_STEP, DeviceTableau
    c = layered_circuit(n, depth, 2, gen_seed=[66, n, depth], circuit_id=17)
    res = {}
    try:
        for mode in (MEASURE_STEP, MEASURE_BLOCKED):
            _mode(ctx, mode)
            t = DeviceTableau(ctx, n, 2).apply_circuit_gates(c)
            out, rnd = t.measure(c.qubits, seed=c.seed, circuit=17)
            res[mode] = (out, rnd, t.export(), t.anomalies())
            t.close()
    finally:
        from paper_2408_00384_amd import MEASURE_AUTO
        _mode(ctx, MEASURE_AUTO)
    a, b = res[MEASURE_STEP], res[MEASURE_BLOCKED]
    assert 0.05 < b[1].mean() < 0.95
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for A, B in zip(a[2], b[2]):
        assert np.array_equal(A, B)
    assert a[3] == 0 and b[3] == 0


def test_large_chunks_fall_back_when_memory_is_short():
    """With the device nearly full (all but 4 GiB held by a torch
    allocation), the blocked pass's chunk scratch at n = 10,000 (about 5.6 GB
    for chunks of 2048) cannot be allocated; the call then takes the
    per-measurement chunk size (about 2.3 GB) and gives the oracle's results;
    cliff_last_error reports the refused allocation."""
    import torch
    from paper_2408_00384_amd import (MEASURE_BLOCKED, CliffError, Context, DeviceTableau, cliff_ctx_set_measure_mode,
                                      cliff_last_error)
    n, shots = 10000, 1
    c = layered_circuit(n, 14, shots, gen_seed=[67, n], circuit_id=18)
    q = np.arange(70, dtype=np.uint32)
    cx = Context(0)
    try:
        cliff_ctx_set_measure_mode(cx.handle, MEASURE_BLOCKED)
        t = DeviceTableau(cx, n, shots).apply_circuit_gates(c)
        torch.cuda.synchronize()
        free, _ = torch.cuda.mem_get_info()
        keep = 4 << 30
        if free <= keep + (1 << 30):
            pytest.skip("less than 5 GiB of device memory free")
        # a known failure first, so that the message checked below is this call's
        with pytest.raises(CliffError):
            cliff_ctx_set_measure_mode(cx.handle, 99)
        assert "measurement scratch" not in cliff_last_error()
        hold = torch.empty(free - keep, dtype=torch.uint8, device="cuda")
        try:
            out, rnd = t.measure(q, seed=c.seed, circuit=18)
        finally:
            del hold
            torch.cuda.empty_cache()
        # the large-chunk allocation was refused and the call recovered
        assert "measurement scratch" in cliff_last_error()
        want_out, want_kinds, tabs = _oracle_run(c, q, shots)
        assert np.array_equal(rnd, want_kinds) and np.array_equal(out, want_out)
        gx, gz, gr = t.export()
        x, z, r = tabs[0]
        assert np.array_equal(gx, x) and np.array_equal(gz, z) and np.array_equal(gr[0], r)
        t.close()
    finally:
        cx.close()

"""cliff_measure_record_noalloc against cliff_measure_record (bit for bit).

Two calls in a row through the C ABI, the second with a smaller input: a
register-resident pass at n = 4,096 (its chunk shrinks to fit the static
scratch, several chunks) and then n = 300 with fewer shots, each compared
with cliff_measure_record on an identical tableau: record bytes, random
flags and the whole tableau afterwards.  Then a measurement past the
register-resident limit (n = 10,241, per-measurement kernels).
"""
import numpy as np
import pytest
import torch

from inputs import layered_circuit

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2408_00384_amd import Context
    c = Context(0)
    yield c
    c.close()


def _both(ctx, c, qubits):
    from paper_2408_00384_amd import DeviceTableau, cliff_measure_record, cliff_measure_record_noalloc
    k = len(qubits)
    res = []
    for fn in (cliff_measure_record, cliff_measure_record_noalloc):
        t = DeviceTableau(ctx, c.n, c.shots).apply_circuit_gates(c)
        rec = torch.full((c.shots, k + 3), 7, dtype=torch.uint8, device="cuda:0")
        rnd = torch.full((k + 3,), 7, dtype=torch.uint8, device="cuda:0")
        torch.cuda.synchronize()
        fn(t.handle, qubits, rec.data_ptr(), k + 3, 2, rnd.data_ptr(), seed=c.seed, circuit=c.circuit_id)
        torch.cuda.synchronize()
        res.append((rec.cpu().numpy(), rnd.cpu().numpy(), t.export(), t.anomalies()))
        t.close()
    return res


@pytest.mark.parametrize("n,shots,k", [(4096, 3, 4096), (300, 2, 120)])
def test_noalloc_equals_measure_record(ctx, n, shots, k):
    c = layered_circuit(n, 12, shots, gen_seed=[80, n], circuit_id=8)
    q = np.concatenate([np.arange(k - 2), [0, 1]]).astype(np.uint32)   # two deterministic repeats
    (ra, da, ta, aa), (rb, db, tb, ab) = _both(ctx, c, q)
    assert np.array_equal(ra, rb) and np.array_equal(da, db)
    assert (ra[:, :2] == 7).all() and (ra[:, -1] == 7).all()   # only columns col0 .. col0 + k - 1 written
    for A, B in zip(ta, tb):
        assert np.array_equal(A, B)
    assert aa == 0 and ab == 0
    assert 0 < int(da[2:-1].sum()) < len(q)


def test_noalloc_past_register_resident_limit(ctx):
    from paper_2408_00384_amd import DeviceTableau, cliff_measure_record, cliff_measure_record_noalloc
    c = layered_circuit(10_241, 4, 1, gen_seed=[81], circuit_id=9)
    q = np.arange(40, dtype=np.uint32)
    outs = []
    for fn in (cliff_measure_record, cliff_measure_record_noalloc):
        t = DeviceTableau(ctx, c.n, 1).apply_circuit_gates(c)
        rec = torch.zeros((1, 40), dtype=torch.uint8, device="cuda:0")
        rnd = torch.zeros(40, dtype=torch.uint8, device="cuda:0")
        fn(t.handle, q, rec.data_ptr(), 40, 0, rnd.data_ptr(), seed=c.seed, circuit=c.circuit_id)
        torch.cuda.synchronize()
        outs.append((rec.cpu().numpy(), rnd.cpu().numpy(), t.export_rows(np.arange(0, 2 * c.n, 97, dtype=np.uint32))))
        t.close()
    (ra, da, xa), (rb, db, xb) = outs
    assert np.array_equal(ra, rb) and np.array_equal(da, db)
    for A, B in zip(xa, xb):
        assert np.array_equal(A, B)

"""ctypes binding of libcliff.so: the C entry points under the same names.

Argument marshalling only; every step of the simulation runs in the library's
HIP kernels.  Device memory comes from torch tensors (plumbing), streams from
torch.cuda.  Importing this module fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libcliff.so")

CLIFF_OK = 0
CLIFF_EINVAL = -1
CLIFF_ENOMEM = -2
CLIFF_EDEVICE = -3
CLIFF_EBUSY = -4
CLIFF_EINTERNAL = -5
OP_H, OP_S, OP_CNOT, OP_SDG, OP_X, OP_Y, OP_Z, OP_CZ, OP_SWAP = range(9)
BASIS_Z, BASIS_X, BASIS_Y = 0, 1, 2


class CliffError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__("%s failed (%d): %s" % (where, code, msg))
        self.code = code


# One HIP runtime per process: PyTorch ships its own copy of the HIP/HSA
# runtime, and a second copy cannot open the device.  Importing torch first
# makes libcliff's libamdhip64.so.7 dependency resolve to the copy already
# loaded, so device memory and streams are shared with torch.
try:
    import torch  # noqa: F401
except ImportError:  # standalone use without PyTorch: /opt/rocm's runtime
    torch = None

if not os.path.exists(LIB_PATH):
    raise ImportError("libcliff.so not built (expected %s); run "
                      "`python paper_2408_00384_amd/build.py`" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_sz = ctypes.c_size_t
_szp = ctypes.POINTER(ctypes.c_size_t)
_vpp = ctypes.POINTER(ctypes.c_void_p)
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64

_SIGS = {
    "cliff_last_error": (ctypes.c_char_p, []),
    "cliff_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "cliff_ctx_create": (ctypes.c_int, [ctypes.c_int, _vp, ctypes.POINTER(_vp)]),
    "cliff_ctx_destroy": (ctypes.c_int, [_vp]),
    "cliff_sync": (ctypes.c_int, [_vp]),
    "cliff_ctx_num_cus": (ctypes.c_int, [_vp]),
    "cliff_calibrate": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "cliff_ctx_set_gate_mode": (ctypes.c_int, [_vp, ctypes.c_int]),
    "cliff_ctx_set_measure_mode": (ctypes.c_int, [_vp, ctypes.c_int]),
    "cliff_ctx_inject_abort": (ctypes.c_int, [_vp, _u64]),
    "cliff_tab_bytes": (_sz, [_u32, _u32]),
    "cliff_tab_bind": (ctypes.c_int, [_vp, _u32, _u32, _vp, _sz, ctypes.POINTER(_vp)]),
    "cliff_tab_unbind": (ctypes.c_int, [_vp]),
    "cliff_tab_info": (ctypes.c_int, [_vp, _u32p, _u32p]),
    "cliff_tab_init_zero": (ctypes.c_int, [_vp]),
    "cliff_apply_gates": (ctypes.c_int, [_vp, _u8p, _u32p, _u32p, _sz]),
    "cliff_apply_layers": (ctypes.c_int, [_vp, _u8p, _u8p, _u32p, _u32p, _u32, _u32]),
    "cliff_encode_layers": (ctypes.c_int, [_u32, _u8p, _u8p, _u32p, _u32p, _u32, _u32, _u64p, _sz,
                                           _u32p, ctypes.POINTER(_sz)]),
    "cliff_apply_encoded": (ctypes.c_int, [_vp, _vp, _u32p, _u32]),
    "cliff_encode_gates": (ctypes.c_int, [_u32, _u8p, _u32p, _u32p, _sz, _u64p, _sz, _u32p, _sz,
                                          ctypes.POINTER(_sz), ctypes.POINTER(_u32)]),
    "cliff_apply_encoded_many": (ctypes.c_int, [_vpp, _vpp, _vpp, _u32p, _sz, ctypes.c_int]),
    "cliff_apply_gates_many": (ctypes.c_int, [_vpp, _vpp, _vpp, _vpp, _szp, _sz, ctypes.c_int]),
    "cliff_measure": (ctypes.c_int, [_vp, _u32p, _sz, _u64, _u64, _u64, _u64, _u8p, _u8p]),
    "cliff_measure_bases": (ctypes.c_int, [_vp, _u32p, _u8p, _sz, _u64, _u64, _u64, _u64, _u8p, _u8p]),
    "cliff_measure_record": (ctypes.c_int, [_vp, _u32p, _sz, _u64, _u64, _u64, _u64, _vp, _sz, _sz, _vp]),
    "cliff_measure_record_noalloc": (ctypes.c_int, [_vp, _u32p, _sz, _u64, _u64, _u64, _u64, _vp, _sz, _sz, _vp]),
    "cliff_reset_record": (ctypes.c_int, [_vp, _u32p, _sz, _u64, _u64, _u64, _u64, _vp, _sz, _sz, _vp]),
    "cliff_apply_cond_paulis": (ctypes.c_int, [_vp, _u32p, _u8p, _u32p, _sz, _vp, _sz]),
    "cliff_sample": (ctypes.c_int, [_vp, _vp, _u32p, _sz, _u64, _u64, _u64, _u8p, _u8p]),
    "cliff_measure_async": (ctypes.c_int, [_vp, _u32p, _sz, _u64, _u64, _u64, _u64]),
    "cliff_tab_read_outcomes": (ctypes.c_int, [_vp, _sz, _u8p, _u8p]),
    "cliff_tab_export": (ctypes.c_int, [_vp, _u8p, _u8p, _u8p]),
    "cliff_tab_export_rows": (ctypes.c_int, [_vp, _u32p, _sz, _u8p, _u8p, _u8p]),
    "cliff_tab_import": (ctypes.c_int, [_vp, _u8p, _u8p, _u8p]),
    "cliff_tab_anomalies": (ctypes.c_int, [_vp, _u64p]),
    "cliff_tab_counters": (ctypes.c_int, [_vp, _u64p]),
    "cliff_tab_reset_counters": (ctypes.c_int, [_vp]),
    "cliff_ctx_profile": (ctypes.c_int, [_vp, ctypes.c_int]),
    "cliff_ctx_profile_read": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _u64p]),
    "cliff_batch_work_bytes": (_sz, []),
    "cliff_batch_run": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _u32, _u64, _vp, _u32, _u32, _u32]),
    "cliff_batch_status": (ctypes.c_int, [_vp, _vp, _u64p]),
    "cliff_batch_order_ops": (ctypes.c_int, [_u32, _u64p, _u32p, _u32]),
    "cliff_graph_begin": (ctypes.c_int, [_vp]),
    "cliff_graph_end": (ctypes.c_int, [_vp, ctypes.POINTER(_vp)]),
    "cliff_graph_launch": (ctypes.c_int, [_vp]),
    "cliff_graph_destroy": (ctypes.c_int, [_vp]),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def exported_symbols():
    """Names of the C entry points this binding declares."""
    return list(_SIGS)


def _check(rc: int, where: str):
    if rc != CLIFF_OK:
        raise CliffError(rc, where, _lib.cliff_last_error().decode(errors="replace"))


def _ptr(a: np.ndarray, t):
    return a.ctypes.data_as(t) if a is not None else None


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# --- the entry points, same names as the C ABI --------------------------------

def cliff_last_error() -> str:
    return _lib.cliff_last_error().decode(errors="replace")


def cliff_strerror(code: int) -> str:
    return _lib.cliff_strerror(code).decode()


def cliff_ctx_create(device: int = 0, stream: int | None = None):
    out = _vp()
    _check(_lib.cliff_ctx_create(device, stream, ctypes.byref(out)), "cliff_ctx_create")
    return out


def cliff_ctx_destroy(ctx):
    _check(_lib.cliff_ctx_destroy(ctx), "cliff_ctx_destroy")


def cliff_sync(ctx):
    _check(_lib.cliff_sync(ctx), "cliff_sync")


def cliff_ctx_num_cus(ctx) -> int:
    return int(_lib.cliff_ctx_num_cus(ctx))


GATES_AUTO, GATES_PER_LAYER, GATES_FUSED = 0, 1, 2
MEASURE_AUTO, MEASURE_STEP, MEASURE_PERSISTENT, MEASURE_BLOCKED = 0, 1, 2, 3


CAL_LDS, CAL_VALU = 0, 1


def cliff_calibrate(ctx, kind: int) -> float:
    """Measured LDS read bytes/s (CAL_LDS) or 32-bit VALU lane ops/s (CAL_VALU)."""
    v = ctypes.c_double()
    _check(_lib.cliff_calibrate(ctx, kind, ctypes.byref(v)), "cliff_calibrate")
    return float(v.value)


def cliff_ctx_set_measure_mode(ctx, mode: int):
    _check(_lib.cliff_ctx_set_measure_mode(ctx, mode), "cliff_ctx_set_measure_mode")


def cliff_ctx_inject_abort(ctx, at: int):
    """The next register-resident pass on ``ctx`` gives up at its measurement
    ``at`` as if a wait had run out (a test aid; 2**64 - 1 cancels)."""
    _check(_lib.cliff_ctx_inject_abort(ctx, at), "cliff_ctx_inject_abort")


def cliff_ctx_set_gate_mode(ctx, mode: int):
    _check(_lib.cliff_ctx_set_gate_mode(ctx, mode), "cliff_ctx_set_gate_mode")


def cliff_tab_bytes(n: int, shots: int) -> int:
    return int(_lib.cliff_tab_bytes(n, shots))


def cliff_tab_bind(ctx, n: int, shots: int, dev_ptr: int, nbytes: int):
    out = _vp()
    _check(_lib.cliff_tab_bind(ctx, n, shots, dev_ptr, nbytes, ctypes.byref(out)), "cliff_tab_bind")
    return out


def cliff_tab_unbind(tab):
    _check(_lib.cliff_tab_unbind(tab), "cliff_tab_unbind")


def cliff_tab_info(tab):
    n, s = _u32(), _u32()
    _check(_lib.cliff_tab_info(tab, ctypes.byref(n), ctypes.byref(s)), "cliff_tab_info")
    return int(n.value), int(s.value)


def cliff_tab_init_zero(tab):
    _check(_lib.cliff_tab_init_zero(tab), "cliff_tab_init_zero")


def cliff_apply_gates(tab, ops, a, b):
    ops, a, b = _arr(ops, np.uint8), _arr(a, np.uint32), _arr(b, np.uint32)
    _check(_lib.cliff_apply_gates(tab, _ptr(ops, _u8p), _ptr(a, _u32p), _ptr(b, _u32p), len(ops)),
           "cliff_apply_gates")


def cliff_apply_layers(tab, h, s, ctrl, tgt):
    h, s = _arr(h, np.uint8), _arr(s, np.uint8)
    ctrl, tgt = _arr(ctrl, np.uint32), _arr(tgt, np.uint32)
    depth = h.shape[0]
    npairs = ctrl.shape[1] if ctrl.ndim == 2 else 0
    _check(_lib.cliff_apply_layers(tab, _ptr(h, _u8p), _ptr(s, _u8p), _ptr(ctrl, _u32p),
                                   _ptr(tgt, _u32p), npairs, depth), "cliff_apply_layers")


def cliff_encode_layers(n, h, s, ctrl, tgt):
    """Returns (ops uint64[nops], offs uint32[depth+1])."""
    h, s = _arr(h, np.uint8), _arr(s, np.uint8)
    ctrl, tgt = _arr(ctrl, np.uint32), _arr(tgt, np.uint32)
    depth = h.shape[0]
    npairs = ctrl.shape[1] if ctrl.ndim == 2 else 0
    offs = np.zeros(depth + 1, np.uint32)
    nops = _sz()
    args = (n, _ptr(h, _u8p), _ptr(s, _u8p), _ptr(ctrl, _u32p), _ptr(tgt, _u32p), npairs, depth)
    _check(_lib.cliff_encode_layers(*args, None, 0, _ptr(offs, _u32p), ctypes.byref(nops)),
           "cliff_encode_layers")
    ops = np.zeros(max(1, nops.value), np.uint64)
    _check(_lib.cliff_encode_layers(*args, _ptr(ops, _u64p), ops.size, _ptr(offs, _u32p),
                                    ctypes.byref(nops)), "cliff_encode_layers")
    return ops[: nops.value], offs


def cliff_encode_gates(n, ops, a, b):
    """Gate list -> (op words uint64[nops], layer offsets uint32[depth+1])."""
    o, a, b = _arr(ops, np.uint8), _arr(a, np.uint32), _arr(b, np.uint32)
    nops, depth = _sz(), _u32()
    args = (n, _ptr(o, _u8p), _ptr(a, _u32p), _ptr(b, _u32p), len(o))
    _check(_lib.cliff_encode_gates(*args, None, 0, None, 0, ctypes.byref(nops), ctypes.byref(depth)),
           "cliff_encode_gates")
    words = np.zeros(max(1, nops.value), np.uint64)
    offs = np.zeros(depth.value + 1, np.uint32)
    _check(_lib.cliff_encode_gates(*args, _ptr(words, _u64p), words.size, _ptr(offs, _u32p), offs.size,
                                   ctypes.byref(nops), ctypes.byref(depth)), "cliff_encode_gates")
    return words[: nops.value], offs


def _ptr_array(items):
    """void* array from handles (c_void_p) or integer addresses."""
    def addr(v):
        if isinstance(v, ctypes.c_void_p):
            return v.value or 0
        return int(v) if v else 0
    return (ctypes.c_void_p * max(1, len(items)))(*[ctypes.c_void_p(addr(v)) for v in items])


def cliff_apply_encoded_many(tabs, dev_ops_ptrs, offs_list, rows_per_group=0):
    """Tableau i runs the device-resident stream dev_ops_ptrs[i] with host offsets offs_list[i]."""
    offs_list = [_arr(o, np.uint32) for o in offs_list]
    depths = np.array([len(o) - 1 for o in offs_list], np.uint32)
    _check(_lib.cliff_apply_encoded_many(_ptr_array(tabs), _ptr_array(dev_ops_ptrs),
                                         _ptr_array([o.ctypes.data for o in offs_list]),
                                         _ptr(depths, _u32p), len(tabs), rows_per_group),
           "cliff_apply_encoded_many")


def cliff_apply_gates_many(tabs, gate_lists, rows_per_group=0):
    """gate_lists[i] = (ops, a, b) for tableau i."""
    lists = [(_arr(o, np.uint8), _arr(a, np.uint32), _arr(b, np.uint32)) for o, a, b in gate_lists]
    counts = np.array([len(o) for o, _, _ in lists], np.uintp)
    _check(_lib.cliff_apply_gates_many(_ptr_array(tabs), _ptr_array([l[0].ctypes.data for l in lists]),
                                       _ptr_array([l[1].ctypes.data for l in lists]),
                                       _ptr_array([l[2].ctypes.data for l in lists]),
                                       counts.ctypes.data_as(_szp), len(tabs), rows_per_group),
           "cliff_apply_gates_many")


def cliff_apply_encoded(tab, dev_ops_ptr: int, offs):
    offs = _arr(offs, np.uint32)
    _check(_lib.cliff_apply_encoded(tab, dev_ops_ptr, _ptr(offs, _u32p), len(offs) - 1),
           "cliff_apply_encoded")


def cliff_measure(tab, qubits, seed=0, circuit=0, shot0=0, m0=0, want_out=True):
    """Returns (outcomes uint8[shots, k] or None, random-flags uint8[k])."""
    _, shots = cliff_tab_info(tab)
    q = _arr(qubits, np.uint32)
    out = np.zeros((shots, len(q)), np.uint8) if want_out else None
    rnd = np.zeros(len(q), np.uint8)
    _check(_lib.cliff_measure(tab, _ptr(q, _u32p), len(q), seed, circuit, shot0, m0,
                              _ptr(out, _u8p), _ptr(rnd, _u8p)), "cliff_measure")
    return out, rnd


def cliff_measure_bases(tab, qubits, bases, seed=0, circuit=0, shot0=0, m0=0, want_out=True):
    """Like cliff_measure with a basis (BASIS_Z / _X / _Y) per measurement."""
    _, shots = cliff_tab_info(tab)
    q = _arr(qubits, np.uint32)
    b = _arr(bases, np.uint8)
    if len(b) != len(q):
        raise ValueError("bases and qubits differ in length")
    out = np.zeros((shots, len(q)), np.uint8) if want_out else None
    rnd = np.zeros(len(q), np.uint8)
    _check(_lib.cliff_measure_bases(tab, _ptr(q, _u32p), _ptr(b, _u8p), len(q), seed, circuit, shot0,
                                    m0, _ptr(out, _u8p), _ptr(rnd, _u8p)), "cliff_measure_bases")
    return out, rnd


def cliff_measure_record(tab, qubits, dev_record_ptr, ld, col0, dev_random_ptr=0, seed=0, circuit=0,
                         shot0=0, m0=0):
    """Outcomes into a device record: shot s, measurement i at [s * ld + col0 + i]."""
    q = _arr(qubits, np.uint32)
    _check(_lib.cliff_measure_record(tab, _ptr(q, _u32p), len(q), seed, circuit, shot0, m0,
                                     dev_record_ptr, ld, col0, dev_random_ptr or None),
           "cliff_measure_record")


def cliff_measure_record_noalloc(tab, qubits, dev_record_ptr, ld, col0, dev_random_ptr=0, seed=0, circuit=0,
                                 shot0=0, m0=0):
    """cliff_measure_record that allocates nothing (the library's static
    device scratch instead of the context's)."""
    q = _arr(qubits, np.uint32)
    _check(_lib.cliff_measure_record_noalloc(tab, _ptr(q, _u32p), len(q), seed, circuit, shot0, m0,
                                             dev_record_ptr, ld, col0, dev_random_ptr or None),
           "cliff_measure_record_noalloc")


def cliff_reset_record(tab, qubits, dev_record_ptr, ld, col0, dev_random_ptr=0, seed=0, circuit=0,
                       shot0=0, m0=0):
    q = _arr(qubits, np.uint32)
    _check(_lib.cliff_reset_record(tab, _ptr(q, _u32p), len(q), seed, circuit, shot0, m0,
                                   dev_record_ptr, ld, col0, dev_random_ptr or None), "cliff_reset_record")


def cliff_apply_cond_paulis(tab, qubits, paulis, cols, dev_record_ptr, ld):
    q, p, c = _arr(qubits, np.uint32), _arr(paulis, np.uint8), _arr(cols, np.uint32)
    if not (len(q) == len(p) == len(c)):
        raise ValueError("qubits, paulis and cols differ in length")
    _check(_lib.cliff_apply_cond_paulis(tab, _ptr(q, _u32p), _ptr(p, _u8p), _ptr(c, _u32p), len(q),
                                        dev_record_ptr, ld), "cliff_apply_cond_paulis")


def cliff_measure_async(tab, qubits, seed=0, circuit=0, shot0=0, m0=0):
    q = _arr(qubits, np.uint32)
    _check(_lib.cliff_measure_async(tab, _ptr(q, _u32p), len(q), seed, circuit, shot0, m0),
           "cliff_measure_async")


def cliff_tab_read_outcomes(tab, k):
    _, shots = cliff_tab_info(tab)
    out = np.zeros((shots, k), np.uint8)
    rnd = np.zeros(k, np.uint8)
    _check(_lib.cliff_tab_read_outcomes(tab, k, _ptr(out, _u8p), _ptr(rnd, _u8p)),
           "cliff_tab_read_outcomes")
    return out, rnd


def cliff_sample(tab, work, qubits, seed=0, circuit=0, shot0=0):
    _, shots = cliff_tab_info(work)
    q = _arr(qubits, np.uint32)
    out = np.zeros((shots, len(q)), np.uint8)
    rnd = np.zeros(len(q), np.uint8)
    _check(_lib.cliff_sample(tab, work, _ptr(q, _u32p), len(q), seed, circuit, shot0,
                             _ptr(out, _u8p), _ptr(rnd, _u8p)), "cliff_sample")
    return out, rnd


def cliff_tab_export(tab):
    """Returns (x uint8[2n, n], z uint8[2n, n], r uint8[shots, 2n])."""
    n, shots = cliff_tab_info(tab)
    x = np.zeros((2 * n, n), np.uint8)
    z = np.zeros((2 * n, n), np.uint8)
    r = np.zeros((shots, 2 * n), np.uint8)
    _check(_lib.cliff_tab_export(tab, _ptr(x, _u8p), _ptr(z, _u8p), _ptr(r, _u8p)), "cliff_tab_export")
    return x, z, r


def cliff_tab_export_rows(tab, rows):
    """Rows `rows` only: (x uint8[k, n], z uint8[k, n], r uint8[shots, k])."""
    n, shots = cliff_tab_info(tab)
    q = _arr(rows, np.uint32)
    k = len(q)
    x = np.zeros((k, n), np.uint8)
    z = np.zeros((k, n), np.uint8)
    r = np.zeros((shots, k), np.uint8)
    _check(_lib.cliff_tab_export_rows(tab, _ptr(q, _u32p), k, _ptr(x, _u8p), _ptr(z, _u8p), _ptr(r, _u8p)),
           "cliff_tab_export_rows")
    return x, z, r


def cliff_tab_import(tab, x, z, r):
    n, shots = cliff_tab_info(tab)
    x = _arr(x, np.uint8).reshape(2 * n, n)
    z = _arr(z, np.uint8).reshape(2 * n, n)
    r = _arr(r, np.uint8).reshape(shots, 2 * n)
    _check(_lib.cliff_tab_import(tab, _ptr(x, _u8p), _ptr(z, _u8p), _ptr(r, _u8p)), "cliff_tab_import")


def cliff_tab_anomalies(tab) -> int:
    v = _u64()
    _check(_lib.cliff_tab_anomalies(tab, ctypes.byref(v)), "cliff_tab_anomalies")
    return int(v.value)


def cliff_tab_counters(tab):
    """dict(anomalies, random, deterministic, alg_bytes): see cliff_tab_counters."""
    out = np.zeros(4, np.uint64)
    _check(_lib.cliff_tab_counters(tab, _ptr(out, _u64p)), "cliff_tab_counters")
    return dict(anomalies=int(out[0]), random=int(out[1]), deterministic=int(out[2]),
                alg_bytes=int(out[3]))


def cliff_tab_reset_counters(tab):
    _check(_lib.cliff_tab_reset_counters(tab), "cliff_tab_reset_counters")


PROF_KINDS = ("gate", "select", "sweep", "final", "other", "batch", "blocked")


def cliff_ctx_profile(ctx, enable: bool):
    _check(_lib.cliff_ctx_profile(ctx, 1 if enable else 0), "cliff_ctx_profile")


def cliff_ctx_profile_read(ctx, kind):
    k = PROF_KINDS.index(kind) if isinstance(kind, str) else int(kind)
    ms = ctypes.c_double()
    n = _u64()
    _check(_lib.cliff_ctx_profile_read(ctx, k, ctypes.byref(ms), ctypes.byref(n)),
           "cliff_ctx_profile_read")
    return float(ms.value), int(n.value)


BATCH_DESC_DTYPE = np.dtype([("n", np.uint32), ("depth", np.uint32), ("shots", np.uint32),
                             ("reserved", np.uint32), ("ops_off", np.uint64), ("offs_off", np.uint64),
                             ("out_off", np.uint64), ("circuit_id", np.uint64)])
BATCH_TEAMS = (64, 128, 256, 512, 1024)   # threads per circuit of the batch kernel
BATCH_MAXN = 256                           # largest batched circuit


def cliff_batch_work_bytes() -> int:
    return int(_lib.cliff_batch_work_bytes())


def cliff_batch_run(ctx, descs_ptr, ops_ptr, offs_ptr, out_ptr, order_ptr, count, seed, work_ptr,
                    team, maxn, max_shots=64):
    _check(_lib.cliff_batch_run(ctx, descs_ptr, ops_ptr, offs_ptr, out_ptr, order_ptr, count, seed,
                                work_ptr, team, maxn, max_shots), "cliff_batch_run")


def cliff_batch_order_ops(n, ops, offs):
    """Reorders each layer of an encoded stream (uint64 ops, in place) for the
    batch kernel's LDS banks; returns ops."""
    if ops.dtype != np.uint64 or not ops.flags.c_contiguous or not ops.flags.writeable:
        raise ValueError("ops must be a writable contiguous uint64 array")
    offs = _arr(offs, np.uint32)
    if len(offs) < 1 or int(offs[-1]) > len(ops):
        raise ValueError("layer offsets past the op stream")
    _check(_lib.cliff_batch_order_ops(n, _ptr(ops, _u64p), _ptr(offs, _u32p), len(offs) - 1),
           "cliff_batch_order_ops")
    return ops


def cliff_batch_status(ctx, work_ptr):
    out = np.zeros(2, np.uint64)
    _check(_lib.cliff_batch_status(ctx, work_ptr, _ptr(out, _u64p)), "cliff_batch_status")
    return dict(rejected=int(out[0]), anomalies=int(out[1]))


def cliff_graph_begin(ctx):
    _check(_lib.cliff_graph_begin(ctx), "cliff_graph_begin")


def cliff_graph_end(ctx):
    out = _vp()
    _check(_lib.cliff_graph_end(ctx, ctypes.byref(out)), "cliff_graph_end")
    return out


def cliff_graph_launch(graph):
    _check(_lib.cliff_graph_launch(graph), "cliff_graph_launch")


def cliff_graph_destroy(graph):
    _check(_lib.cliff_graph_destroy(graph), "cliff_graph_destroy")


__all__ = [n for n in list(globals()) if n.startswith("cliff_")] + [
    "CLIFF_OK", "CLIFF_EINVAL", "CLIFF_ENOMEM", "CLIFF_EDEVICE", "CLIFF_EBUSY",
    "CLIFF_EINTERNAL", "OP_H", "OP_S", "OP_CNOT", "OP_SDG", "OP_X", "OP_Y", "OP_Z", "OP_CZ",
    "OP_SWAP", "BASIS_Z", "BASIS_X", "BASIS_Y", "CliffError", "LIB_PATH", "exported_symbols",
    "PROF_KINDS", "BATCH_DESC_DTYPE", "BATCH_TEAMS", "BATCH_MAXN", "GATES_AUTO", "GATES_PER_LAYER",
    "GATES_FUSED", "MEASURE_AUTO", "MEASURE_STEP", "MEASURE_PERSISTENT", "MEASURE_BLOCKED", "CAL_LDS", "CAL_VALU"]

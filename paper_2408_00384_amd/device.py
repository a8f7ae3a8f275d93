"""Device memory and stream plumbing around the C ABI (PyTorch allocations only).

``Context`` wraps one cliff_ctx bound to a torch (HIP) stream; ``DeviceTableau``
owns a torch uint8 buffer of cliff_tab_bytes(n, shots) bytes and the tableau
view bound onto it.  Nothing here computes anything about the tableau.
"""
from __future__ import annotations

import torch

from . import _binding as B


class Context:
    def __init__(self, device: int = 0, stream: "torch.cuda.Stream | None" = None):
        if not torch.cuda.is_available():
            raise RuntimeError("paper_2408_00384_amd needs a ROCm GPU; none is visible")
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.handle = B.cliff_ctx_create(device, self.stream.cuda_stream)

    def sync(self):
        B.cliff_sync(self.handle)

    @property
    def num_cus(self) -> int:
        return B.cliff_ctx_num_cus(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            B.cliff_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceTableau:
    """A tableau of n qubits with `shots` sign columns in a torch-owned buffer."""

    def __init__(self, ctx: Context, n: int, shots: int = 1, init: bool = True):
        self.ctx = ctx
        self.n, self.shots = int(n), int(shots)
        self.nbytes = B.cliff_tab_bytes(self.n, self.shots)
        if self.nbytes == 0:
            raise ValueError("invalid tableau size n=%d shots=%d" % (n, shots))
        self.buf = torch.empty(self.nbytes + 256, dtype=torch.uint8,
                               device="cuda:%d" % ctx.device)
        ptr = self.buf.data_ptr()
        self.ptr = (ptr + 255) & ~255
        self.handle = B.cliff_tab_bind(ctx.handle, self.n, self.shots, self.ptr, self.nbytes)
        if init:
            self.init_zero()

    def init_zero(self):
        B.cliff_tab_init_zero(self.handle)
        return self

    def apply_layers(self, h, s, ctrl, tgt):
        B.cliff_apply_layers(self.handle, h, s, ctrl, tgt)
        return self

    def apply_circuit_gates(self, c):
        return self.apply_layers(c.h, c.s, c.ctrl, c.tgt)

    def apply_gates(self, ops, a, b):
        B.cliff_apply_gates(self.handle, ops, a, b)
        return self

    def measure(self, qubits, seed=0, circuit=0, shot0=0, m0=0):
        return B.cliff_measure(self.handle, qubits, seed, circuit, shot0, m0)

    def measure_bases(self, qubits, bases, seed=0, circuit=0, shot0=0, m0=0):
        return B.cliff_measure_bases(self.handle, qubits, bases, seed, circuit, shot0, m0)

    def export(self):
        return B.cliff_tab_export(self.handle)

    def export_rows(self, rows):
        return B.cliff_tab_export_rows(self.handle, rows)

    def import_(self, x, z, r):
        B.cliff_tab_import(self.handle, x, z, r)
        return self

    def anomalies(self) -> int:
        return B.cliff_tab_anomalies(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            B.cliff_tab_unbind(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

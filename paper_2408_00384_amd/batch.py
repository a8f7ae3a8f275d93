"""Batched execution of many small circuits (device plumbing around cliff_batch_run).

A ``BatchPlan`` packs circuits into one device-resident op stream with one
descriptor per circuit, splits them into size buckets (max n 64 / 128 / 256),
orders each bucket by estimated cost (largest first, so the device work queue
ends with short circuits), and runs every bucket as one persistent launch with
the team size the autotuner chose for it.  The whole sequence can be captured
once into a HIP graph and replayed.  All simulation work runs in the
library's batch kernel; this module only marshals arrays.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import _binding as B

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_PATH = os.path.join(HERE, "tuning", "batch_gfx950.json")
BUCKETS = (64, 128, 256)
DEFAULT_TEAM = {64: 64, 128: 128, 256: 256}


def load_tuning(path: str = TUNING_PATH) -> dict:
    """{maxn: team} from the autotuner's table, or the defaults."""
    table = dict(DEFAULT_TEAM)
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
        for k, v in rec.get("best", {}).items():
            table[int(k)] = int(v["team"])
    return table


def bucket_of(n: int) -> int:
    for b in BUCKETS:
        if n <= b:
            return b
    raise ValueError("batched circuits need n <= %d (got %d)" % (BUCKETS[-1], n))


def circuit_cost(n: int, depth: int) -> float:
    # gate sweeps ~ depth * n * words, measurement ~ n * n * words
    return float(n) * (depth + n) * ((2 * n + 63) // 64)


class BatchPlan:
    def __init__(self, ctx, circuits, seed=None, teams=None, device="cuda:0"):
        if not circuits:
            raise ValueError("empty batch")
        self.ctx = ctx
        self.circuits = circuits
        self.seed = int(circuits[0].seed if seed is None else seed)
        self.teams = dict(load_tuning() if teams is None else teams)
        count = len(circuits)
        descs = np.zeros(count, dtype=B.BATCH_DESC_DTYPE)
        ops_parts, offs_parts = [], []
        # per circuit: op words and those with a two-qubit gate (for traffic accounting)
        self.op_count = np.zeros(count, np.int64)
        self.pair_count = np.zeros(count, np.int64)
        ops_off = offs_off = out_off = 0
        for i, c in enumerate(circuits):
            if c.shots < 1 or c.shots > 64:
                raise ValueError("batched circuits need 1..64 shots")
            if len(c.qubits) != c.n or not np.array_equal(c.qubits, np.arange(c.n)):
                raise ValueError("batched circuits measure qubits 0..n-1 in order")
            ops, offs = B.cliff_encode_layers(c.n, c.h, c.s, c.ctrl, c.tgt)
            self.op_count[i] = len(ops)
            self.pair_count[i] = int(np.count_nonzero(ops >> np.uint64(62)))
            descs[i] = (c.n, c.depth, c.shots, 0, ops_off, offs_off, out_off, c.circuit_id)
            ops_parts.append(ops)
            offs_parts.append(offs)
            ops_off += len(ops)
            offs_off += len(offs)
            out_off += c.shots * c.n
        self.out_bytes = out_off
        ops_all = np.concatenate(ops_parts) if ops_off else np.zeros(1, np.uint64)
        offs_all = np.concatenate(offs_parts)
        self.d_descs = torch.from_numpy(descs.view(np.uint8).copy()).to(device)
        self.d_ops = torch.from_numpy(np.ascontiguousarray(ops_all).view(np.int64)).to(device)
        self.d_offs = torch.from_numpy(offs_all.view(np.int32).copy()).to(device)
        self.d_out = torch.zeros(max(1, out_off), dtype=torch.uint8, device=device)
        self.descs = descs
        # buckets, each ordered by decreasing cost
        self.buckets = []
        ns = descs["n"].astype(np.int64)
        depths = descs["depth"].astype(np.int64)
        for b in BUCKETS:
            lo = 0 if b == BUCKETS[0] else BUCKETS[BUCKETS.index(b) - 1]
            idx = np.nonzero((ns > lo) & (ns <= b))[0]
            if len(idx) == 0:
                continue
            cost = np.array([circuit_cost(ns[i], depths[i]) for i in idx])
            idx = idx[np.argsort(-cost, kind="stable")].astype(np.uint32)
            order = torch.from_numpy(idx.view(np.int32).copy()).to(device)
            self.buckets.append((b, len(idx), order))
        # one device scratch slot (queue head, error counters) per bucket launch
        self.work_stride = B.cliff_batch_work_bytes()
        self.d_work = torch.zeros(self.work_stride * max(1, len(self.buckets)), dtype=torch.uint8,
                                  device=device)
        self.graph = None
        # uploads ran on torch's current stream; the batch kernels run on the
        # context's stream, which waits for them (no device-wide sync)
        cur = torch.cuda.current_stream()
        if cur != ctx.stream:
            ctx.stream.wait_stream(cur)

    def launch(self):
        """Enqueue every bucket on the context stream (no host sync)."""
        for k, (maxn, cnt, order) in enumerate(self.buckets):
            B.cliff_batch_run(self.ctx.handle, self.d_descs.data_ptr(), self.d_ops.data_ptr(),
                              self.d_offs.data_ptr(), self.d_out.data_ptr(), order.data_ptr(), cnt,
                              self.seed, self.d_work.data_ptr() + k * self.work_stride,
                              self.teams[maxn], maxn)

    def capture(self):
        """Capture the launches into a HIP graph (context must use a side stream)."""
        B.cliff_graph_begin(self.ctx.handle)
        try:
            self.launch()
        finally:
            self.graph = B.cliff_graph_end(self.ctx.handle)
        return self

    def run(self):
        if self.graph is not None:
            B.cliff_graph_launch(self.graph)
        else:
            self.launch()
        return self

    def status(self):
        tot = dict(rejected=0, anomalies=0)
        for k in range(len(self.buckets)):
            st = B.cliff_batch_status(self.ctx.handle, self.d_work.data_ptr() + k * self.work_stride)
            for key in tot:
                tot[key] += st[key]
        return tot

    def outcomes(self):
        """List of uint8 [shots, n] outcome arrays, one per circuit (synchronizes)."""
        self.ctx.sync()
        with torch.cuda.stream(self.ctx.stream):   # copy on this plan's stream only
            host = self.d_out.cpu().numpy()
        res = []
        for d in self.descs:
            o, s, n = int(d["out_off"]), int(d["shots"]), int(d["n"])
            res.append(host[o:o + s * n].reshape(s, n))
        return res

    def close(self):
        if self.graph is not None:
            B.cliff_graph_destroy(self.graph)
            self.graph = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

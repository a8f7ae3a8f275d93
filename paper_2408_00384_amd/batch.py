"""Batched execution of many small circuits (device plumbing around cliff_batch_run).

A ``BatchPlan`` packs circuits into one device-resident op stream with one
descriptor per circuit, splits them into size buckets by n (bucket edges and
the team size of each bucket from the autotuner's table), orders each bucket by
estimated cost (largest first, so the device work queue ends with short
circuits), and runs every bucket as one persistent launch whose LDS is sized
for the bucket's largest circuit and most shots.  The whole sequence can be
captured once into a HIP graph and replayed.  All simulation work runs in the
library's batch kernel; this module only marshals arrays.
"""
from __future__ import annotations

import concurrent.futures as cf
import json
import os

import numpy as np
import torch

from . import _binding as B

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_PATH = os.path.join(HERE, "tuning", "batch_gfx950.json")
DEFAULT_TEAMS = {64: 128, 128: 256, 256: 256}   # bucket edge (largest n) -> team


def load_tuning(path: str = TUNING_PATH) -> dict:
    """{bucket edge: team} from the autotuner's table, or the defaults.  The
    edges are the largest n of each bucket, ascending; the last is 256."""
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
        best = rec.get("best", {})
        if best:
            return check_teams({int(k): int(v["team"]) for k, v in best.items()})
    return dict(DEFAULT_TEAMS)


def check_teams(teams: dict) -> dict:
    for edge, team in teams.items():
        if not 1 <= edge <= B.BATCH_MAXN or team not in B.BATCH_TEAMS:
            raise ValueError("bad bucket %d -> team %d" % (edge, team))
    return dict(sorted(teams.items()))


def circuit_cost(n: int, depth: int) -> float:
    # gate sweeps ~ depth * n * words, measurement ~ n * n * words
    return float(n) * (depth + n) * ((2 * n + 63) // 64)


class BatchPlan:
    def __init__(self, ctx, circuits, seed=None, teams=None, device="cuda:0", encoded=None):
        """teams: {bucket edge: team}, edges ascending (circuit n <= edge
        goes to the first such bucket), default the autotuner's table.
        encoded: optional list of (ops, offs) from cliff_encode_layers, one
        per circuit, to skip re-encoding."""
        if not circuits:
            raise ValueError("empty batch")
        self.ctx = ctx
        self.circuits = circuits
        self.seed = int(circuits[0].seed if seed is None else seed)
        self.teams = check_teams(load_tuning() if teams is None else teams)
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
            ops, offs = (B.cliff_encode_layers(c.n, c.h, c.s, c.ctrl, c.tgt) if encoded is None
                         else encoded[i])
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
        # each circuit's layers in the order that spreads the kernel's LDS
        # accesses over distinct banks (same results in any order); circuits
        # on host threads (the library call releases the interpreter lock)
        def order(d):
            o, f, depth = int(d["ops_off"]), int(d["offs_off"]), int(d["depth"])
            if int(offs_all[f + depth]):
                B.cliff_batch_order_ops(int(d["n"]), ops_all[o: o + int(offs_all[f + depth])],
                                        offs_all[f: f + depth + 1])
        if count >= 64:
            with cf.ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
                list(ex.map(order, descs))
        else:
            for d in descs:
                order(d)
        self.d_descs = torch.from_numpy(descs.view(np.uint8).copy()).to(device)
        self.d_ops = torch.from_numpy(np.ascontiguousarray(ops_all).view(np.int64)).to(device)
        self.d_offs = torch.from_numpy(offs_all.view(np.int32).copy()).to(device)
        self.d_out = torch.zeros(max(1, out_off), dtype=torch.uint8, device=device)
        self.descs = descs
        # buckets, each ordered by decreasing cost, with the LDS bounds of its
        # contents (largest n, most shots)
        self.buckets = []
        ns = descs["n"].astype(np.int64)
        depths = descs["depth"].astype(np.int64)
        shots = descs["shots"].astype(np.int64)
        if ns.max() > max(self.teams):
            raise ValueError("circuit with n = %d above the largest bucket (%d)" % (ns.max(), max(self.teams)))
        lo = 0
        for edge, team in self.teams.items():
            idx = np.nonzero((ns > lo) & (ns <= edge))[0]
            lo = edge
            if len(idx) == 0:
                continue
            cost = np.array([circuit_cost(ns[i], depths[i]) for i in idx])
            idx = idx[np.argsort(-cost, kind="stable")].astype(np.uint32)
            order = torch.from_numpy(idx.view(np.int32).copy()).to(device)
            self.buckets.append(dict(edge=edge, team=team, count=len(idx), order=order,
                                     maxn=int(ns[idx].max()), max_shots=int(shots[idx].max())))
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
        for k, b in enumerate(self.buckets):
            B.cliff_batch_run(self.ctx.handle, self.d_descs.data_ptr(), self.d_ops.data_ptr(),
                              self.d_offs.data_ptr(), self.d_out.data_ptr(), b["order"].data_ptr(),
                              b["count"], self.seed, self.d_work.data_ptr() + k * self.work_stride,
                              b["team"], b["maxn"], b["max_shots"])

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

"""Continuous-batching request server for Clifford circuits on one GPU.

Requests (a layered circuit measured on every qubit, with a shot count)
arrive over time.  The server admits them first come, first served as device
memory and execution lanes free up, so work of requests that arrive while
others run is enqueued right away and overlaps on the device:

  * memory: every admitted request holds its device bytes in one arena of a
    fixed budget: on an HBM lane its tableau (cliff_tab_bytes(n, shots)); on
    the batch lane, whose tableaux live in LDS, what the batched launch keeps
    for it in device memory (its op stream, layer offsets, descriptor and
    outcome bytes, request_bytes below).  A request waits until its bytes
    fit; one larger than the whole budget is rejected.  Each HBM lane's
    context also keeps the register-resident measurement's chunk scratch,
    sized once by the largest tableau shape the lane has measured (about
    270 MB at n = 4,096); it is not charged per request;
  * HBM lanes: requests that do not fit the batched kernel (n > 256 or more
    than 64 shots) run on one of several streams, each with its own context:
    tableau bound inside the arena, |0...0>, all gate layers, then all
    measurements for all shots at once (the tableau stays on the device across
    shots: the shots are sign columns of the one tableau);
  * batch lane: waiting small requests are gathered into one persistent
    batched launch whenever that lane is free.

All simulation work happens in libcliff's kernels; this module only decides
what to enqueue where and when, and keeps time.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np
import torch

from . import _binding as B
from .batch import BatchPlan
from .device import Context

ALIGN = 256


class ArenaAllocator:
    """First-fit allocator of byte ranges in [0, size) (host bookkeeping only)."""

    def __init__(self, size: int):
        self.size = int(size)
        self.free_list = [(0, self.size)]   # sorted (offset, length)
        self.used = 0
        self.peak = 0

    def alloc(self, nbytes: int):
        need = (int(nbytes) + ALIGN - 1) // ALIGN * ALIGN
        for i, (off, ln) in enumerate(self.free_list):
            if ln >= need:
                if ln == need:
                    self.free_list.pop(i)
                else:
                    self.free_list[i] = (off + need, ln - need)
                self.used += need
                self.peak = max(self.peak, self.used)
                return off, need
        return None

    def free(self, off: int, need: int):
        self.used -= need
        fl = self.free_list
        fl.append((off, need))
        fl.sort()
        merged = []
        for o, ln in fl:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free_list = merged


@dataclasses.dataclass
class Result:
    rid: int
    n: int
    shots: int
    arrival: float
    admitted: float = 0.0
    done: float = 0.0
    path: str = ""
    outcomes: np.ndarray | None = None
    random: np.ndarray | None = None
    error: str | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def batch_request_bytes(c) -> int:
    """Device bytes the batched launch keeps for circuit c: op words (at most
    one per gate; runs of single-qubit gates are composed), layer offsets,
    a descriptor, and the outcome bytes, rounded up as the arena rounds."""
    raw = 8 * c.gate_count() + 4 * (c.depth + 1) + 48 + c.shots * c.n
    return (raw + ALIGN - 1) // ALIGN * ALIGN


def request_bytes(c, batch: bool) -> int:
    return batch_request_bytes(c) if batch else B.cliff_tab_bytes(c.n, c.shots)


class _Lane:
    def __init__(self, device: int):
        self.stream = torch.cuda.Stream(device)
        self.ctx = Context(device, self.stream)
        self.job = None


class Server:
    def __init__(self, budget_bytes: int = 64 << 30, lanes: int = 8, batch_max: int = 512,
                 small_n: int = 256, small_shots: int = 64, device: int = 0,
                 use_batch_lane: bool = True):
        self.device = device
        self.budget = int(budget_bytes)
        self.arena = torch.empty(self.budget, dtype=torch.uint8, device="cuda:%d" % device)
        self.base = (self.arena.data_ptr() + ALIGN - 1) // ALIGN * ALIGN
        self.alloc = ArenaAllocator(self.budget - (self.base - self.arena.data_ptr()))
        self.lanes = [_Lane(device) for _ in range(lanes)]
        self.batch_lane = _Lane(device) if use_batch_lane else None
        self.batch_max = batch_max
        self.small_n, self.small_shots = small_n, small_shots
        self.queue = collections.deque()
        self.results = {}
        self.t0 = None

    # ------------------------------------------------------------------ util
    def now(self) -> float:
        return time.perf_counter() - self.t0

    def _small(self, c) -> bool:
        return (self.batch_lane is not None and c.n <= self.small_n and c.shots <= self.small_shots)

    # --------------------------------------------------------------- launch
    def _launch_hbm(self, lane, rid, c, res):
        nbytes = B.cliff_tab_bytes(c.n, c.shots)
        got = self.alloc.alloc(nbytes)
        if got is None:
            return False
        off, need = got
        tab = B.cliff_tab_bind(lane.ctx.handle, c.n, c.shots, self.base + off, need)
        B.cliff_tab_init_zero(tab)
        B.cliff_apply_layers(tab, c.h, c.s, c.ctrl, c.tgt)
        B.cliff_measure_async(tab, c.qubits, c.seed, c.circuit_id, 0, 0)
        ev = torch.cuda.Event()
        ev.record(lane.stream)
        res.admitted, res.path = self.now(), "hbm"
        lane.job = ("hbm", ev, [(rid, tab, off, need)])
        return True

    def _launch_batch(self, lane):
        take = []
        held = []
        rest = collections.deque()
        while self.queue and len(take) < self.batch_max:
            rid = self.queue.popleft()
            c = self.requests[rid]
            if not self._small(c):
                rest.append(rid)
                continue
            need = request_bytes(c, batch=True)
            if need > self.alloc.size:
                res = self.results[rid]
                res.error = "request of %d bytes exceeds the budget" % need
                res.done = self.now()
                continue
            got = self.alloc.alloc(need)
            if got is None:
                rest.append(rid)
                break
            take.append(rid)
            held.append(got)
        rest.extend(self.queue)
        self.queue = rest
        if not take:
            return
        with torch.cuda.stream(lane.stream):
            plan = BatchPlan(lane.ctx, [self.requests[r] for r in take])
            plan.run()
        ev = torch.cuda.Event()
        ev.record(lane.stream)
        t = self.now()
        for r in take:
            self.results[r].admitted, self.results[r].path = t, "batch"
        lane.job = ("batch", ev, (take, held, plan))

    def _schedule(self):
        # batch lane: all waiting small requests at once
        if self.batch_lane is not None and self.batch_lane.job is None and \
                any(self._small(self.requests[r]) for r in self.queue):
            self._launch_batch(self.batch_lane)
        # HBM lanes: first come, first served
        for lane in self.lanes:
            if lane.job is not None:
                continue
            # small requests wait for the batch lane; take the first other one
            pick = None
            for r in self.queue:
                if not self._small(self.requests[r]):
                    pick = r
                    break
            if pick is None:
                return
            c = self.requests[pick]
            if B.cliff_tab_bytes(c.n, c.shots) > self.alloc.size:
                self.queue.remove(pick)
                res = self.results[pick]
                res.error = "tableau of %d bytes exceeds the budget" % B.cliff_tab_bytes(c.n, c.shots)
                res.done = self.now()
                continue
            if not self._launch_hbm(lane, pick, c, self.results[pick]):
                return   # wait for memory
            self.queue.remove(pick)

    def _poll(self):
        progressed = False
        for lane in self.lanes + ([self.batch_lane] if self.batch_lane is not None else []):
            if lane.job is None or not lane.job[1].query():
                continue
            kind, ev, payload = lane.job
            t = self.now()
            if kind == "hbm":
                for rid, tab, off, need in payload:
                    c = self.requests[rid]
                    out, rnd = B.cliff_tab_read_outcomes(tab, len(c.qubits))
                    res = self.results[rid]
                    res.outcomes, res.random, res.done = out, rnd, t
                    B.cliff_tab_unbind(tab)
                    self.alloc.free(off, need)
            else:
                take, held, plan = payload
                outs = plan.outcomes()
                for r, o, (off, need) in zip(take, outs, held):
                    res = self.results[r]
                    res.outcomes, res.done = o, t
                    self.alloc.free(off, need)
                plan.close()
            lane.job = None
            progressed = True
        return progressed

    # ------------------------------------------------------------------ run
    def run(self, circuits, arrivals, realtime: bool = True, one_at_a_time: bool = False):
        """Serve circuits[i] arriving at arrivals[i] seconds.  Returns results by id.

        realtime=False admits every request at once (closed loop);
        one_at_a_time=True runs each request alone, the next one admitted only
        after the previous finished."""
        self.requests = list(circuits)
        order = np.argsort(np.asarray(arrivals, dtype=float), kind="stable")
        self.results = {i: Result(i, c.n, c.shots, float(arrivals[i])) for i, c in enumerate(circuits)}
        self.queue.clear()
        torch.cuda.synchronize()
        self.t0 = time.perf_counter()
        nxt = 0
        done = 0
        total = len(circuits)
        while done < total:
            now = self.now()
            while nxt < total and (not realtime or arrivals[order[nxt]] <= now) and \
                    (not one_at_a_time or (not self.queue and self._idle())):
                r = int(order[nxt])
                if not realtime:
                    self.results[r].arrival = now
                self.queue.append(r)
                nxt += 1
            self._schedule()
            progressed = self._poll()
            done = sum(1 for r in self.results.values() if r.done > 0)
            if not progressed:
                time.sleep(20e-6)
        return self.results

    def _idle(self) -> bool:
        lanes = self.lanes + ([self.batch_lane] if self.batch_lane is not None else [])
        return all(l.job is None for l in lanes)

    def close(self):
        for lane in self.lanes + ([self.batch_lane] if self.batch_lane is not None else []):
            lane.ctx.close()


def summarize(results, wall_s: float | None = None):
    ok = [r for r in results.values() if r.error is None]
    lat = np.array([r.latency for r in ok]) * 1e3
    first = min(r.arrival for r in results.values())
    last = max(r.done for r in results.values())
    span = wall_s if wall_s is not None else (last - first)
    return {
        "requests": len(results), "completed": len(ok),
        "rejected": len(results) - len(ok),
        "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_ms": float(lat.mean()) if len(lat) else None,
        "circuits_per_s": len(ok) / span if span > 0 else None,
        "paths": {p: sum(1 for r in ok if r.path == p) for p in ("hbm", "batch")},
    }

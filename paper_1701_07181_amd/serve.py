"""Continuous-batching request server for transformed Radau IIA solves.

Requests arrive over time (Poisson arrivals in the benchmark).  A request
carries an operator (BSR Jacobian, mass blocks, dt, stage count; already in
device memory) and a right-hand side; some re-use an operator whose
factorization is still resident.  Two host threads share the device:

  * the preparation thread sets up and factors new operators on a side
    stream (admission by device-memory budget: an operator waits until its
    workspace fits, evicting idle resident factorizations, least recently
    used first); re-used operators need no preparation;
  * the main loop keeps one `Batch` iterating on its own stream: between
    GMRES cycles it admits prepared requests into free slots (a member
    joins at the next cycle boundary, so new work overlaps the members
    already iterating), advances every member by one cycle, and retires the
    finished ones, recording arrival-to-completion latency.

All numerics run in libirk; this module only schedules.
"""
from __future__ import annotations

import collections
import dataclasses
import queue
import threading
import time
from typing import Dict, List, Optional

import numpy as np
import torch

from . import Batch, Options, Solver, OK


@dataclasses.dataclass
class Request:
    rid: int
    op_id: int                 # operator identity (re-used operators share it)
    system: object             # s, T, m, nJ, dt, row_ptr, col_idx (host), J, M (device tensors)
    rhs: torch.Tensor          # device vector
    arrival: float             # seconds after the start of the run


@dataclasses.dataclass
class Result:
    rid: int
    op_id: int
    x: torch.Tensor
    info: dict
    arrival: float
    done: float
    reused: bool


class Server:
    def __init__(self, options: Options, capacity: int = 64, max_elements: int = 1 << 20,
                 budget_bytes: int = 96 << 30, device: Optional[torch.device] = None):
        self.options = options
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.Stream(self.device)        # batch iteration
        self.side = torch.cuda.Stream(self.device)          # setup + factorization
        self.batch = Batch(capacity, max_elements, device=self.device, stream=self.stream)
        self.capacity = capacity
        self.budget = budget_bytes
        self.lock = threading.Lock()
        self.resident: "collections.OrderedDict[int, Solver]" = collections.OrderedDict()
        self.busy: Dict[int, bool] = {}                     # op_id -> member in the batch
        self.bytes_of: Dict[int, int] = {}
        self.reserved = 0
        self.prep_q: "queue.Queue" = queue.Queue()
        self.ready: collections.deque = collections.deque()
        self.active: Dict[int, tuple] = {}                  # rid -> (request, reused)
        self.results: List[Result] = []
        self.stalls = 0                                     # waits for memory or a free slot
        self.evictions = 0                                  # resident factorizations dropped
        self.t0 = time.perf_counter()
        self.error: Optional[BaseException] = None
        self.worker = threading.Thread(target=self._prep_loop, daemon=True)
        self.worker.start()

    # -- device-memory budget --
    def _estimate(self, sy) -> int:
        n = sy.s * sy.T * sy.m
        blocks = (sy.nJ * int(len(sy.col_idx)) + sy.T) * sy.m * sy.m
        return int(8 * (5 * blocks + (self.options.restart + 12) * n))

    def _reserve(self, need: int) -> bool:
        with self.lock:
            used = sum(self.bytes_of.values()) + self.reserved
            while used + need > self.budget:
                victim = next((k for k in self.resident if not self.busy.get(k, False)), None)
                if victim is None:
                    return False
                self.resident.pop(victim).close()
                used -= self.bytes_of.pop(victim)
                self.evictions += 1
            self.reserved += need
            return True

    # -- preparation thread --
    def _prep_loop(self):
        torch.cuda.set_device(self.device)
        try:
            while True:
                req = self.prep_q.get()
                if req is None:
                    return
                with self.lock:
                    solver = self.resident.get(req.op_id)
                if solver is not None:
                    self.ready.append((req, True))
                    continue
                need = self._estimate(req.system)
                while not self._reserve(need):
                    self.stalls += 1
                    time.sleep(0.0005)
                with torch.cuda.stream(self.side):
                    solver = Solver(req.system, self.options, device=self.device, stream=self.side)
                    solver.factor()
                self.side.synchronize()         # factors complete before the batch stream reads them
                with self.lock:
                    self.reserved -= need
                    self.resident[req.op_id] = solver
                    self.bytes_of[req.op_id] = solver.workspace_bytes
                self.ready.append((req, False))
        except BaseException as e:      # surfaced by the main loop
            self.error = e

    # -- main loop --
    def _admit_ready(self):
        skipped = collections.deque()
        while self.ready and len(self.active) < self.capacity:
            req, reused = self.ready.popleft()
            with self.lock:
                if self.busy.get(req.op_id, False):
                    skipped.append((req, reused))      # its handle is still iterating
                    continue
                solver = self.resident[req.op_id]
                self.resident.move_to_end(req.op_id)
                self.busy[req.op_id] = True
            st = self.batch.admit(solver, req.rhs, tag=req.rid)
            if st != OK:
                with self.lock:
                    self.busy[req.op_id] = False
                skipped.append((req, reused))
                self.stalls += 1
                break
            self.active[req.rid] = (req, reused)
        while skipped:
            self.ready.appendleft(skipped.pop())

    def step(self):
        if self.error:
            raise self.error
        self._admit_ready()
        if self.active:
            self.batch.advance(1)
        for tag, x, info in self.batch.retire():
            req, reused = self.active.pop(tag)
            with self.lock:
                self.busy[req.op_id] = False
            self.results.append(Result(req.rid, req.op_id, x, info, req.arrival,
                                       time.perf_counter() - self.t0, reused))

    def run(self, requests: List[Request]) -> List[Result]:
        """Replay requests at their arrival times until all have completed."""
        torch.cuda.synchronize(self.device)     # right-hand sides written on other streams
        self.t0 = time.perf_counter()
        pending = sorted(requests, key=lambda r: r.arrival)
        k = 0
        while k < len(pending) or len(self.results) < len(pending):
            now = time.perf_counter() - self.t0
            while k < len(pending) and pending[k].arrival <= now:
                self.prep_q.put(pending[k])
                k += 1
            if not self.active and not self.ready:
                time.sleep(0.0002)
                if self.error:
                    raise self.error
                continue
            self.step()
        return self.results

    def close(self):
        self.prep_q.put(None)
        self.worker.join(timeout=60)
        self.batch.close()
        for s in self.resident.values():
            s.close()
        self.resident.clear()


def latency_stats(results: List[Result]) -> dict:
    lat = np.array([r.done - r.arrival for r in results])
    span = max(r.done for r in results) - min(r.arrival for r in results)
    return {"n": len(results), "solves_per_s": len(results) / span if span > 0 else float("nan"),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_iters": float(np.mean([r.info["iters"] for r in results])),
            "converged": int(sum(r.info["converged"] for r in results)),
            "reused": int(sum(r.reused for r in results))}

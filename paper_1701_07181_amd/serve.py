"""Continuous-batching request server for transformed Radau IIA solves.

Requests arrive over time (Poisson arrivals in the benchmark).  A request
carries an operator (BSR Jacobian, mass blocks, dt, stage count; already in
device memory) and a right-hand side; some re-use an operator whose
factorization is still resident.  Two host threads share the device:

  * the preparation thread sets up and factors new operators on a side
    stream, all operators that arrived since its last round together (one
    batched factorization: each level of every operator in the same
    launches); re-used operators need no preparation.  Admission is by device
    memory: every operator's workspace is a range of one pool allocated when
    the server starts (its memory budget), so serving itself never calls the
    device allocator.  An operator waits until a range of its size is free,
    evicting idle resident factorizations, least recently used first;
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

from . import Batch, Options, Solver, OK, factor_batched


class _NoRoom(Exception):
    """No pool range fits now and the caller asked not to wait."""


class WorkspacePool:
    """First-fit ranges of one device allocation (offsets 256-byte aligned,
    free neighbours merged).  Not thread-safe: the server holds its lock."""

    ALIGN = 256

    def __init__(self, nbytes: int, device: torch.device):
        self.size = self.round(nbytes)
        self.mem = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free: List[List[int]] = [[0, self.size]]      # [offset, bytes], ascending offsets

    @classmethod
    def round(cls, n: int) -> int:
        return (int(n) + cls.ALIGN - 1) // cls.ALIGN * cls.ALIGN

    def take(self, nbytes: int) -> Optional[int]:
        n = self.round(nbytes)
        for q, (off, size) in enumerate(self.free):
            if size >= n:
                if size == n:
                    del self.free[q]
                else:
                    self.free[q] = [off + n, size - n]
                return off
        return None

    def give(self, off: int, nbytes: int):
        n = self.round(nbytes)
        q = 0
        while q < len(self.free) and self.free[q][0] < off:
            q += 1
        self.free.insert(q, [off, n])
        if q + 1 < len(self.free) and off + n == self.free[q + 1][0]:
            self.free[q][1] += self.free.pop(q + 1)[1]
        if q > 0 and self.free[q - 1][0] + self.free[q - 1][1] == off:
            self.free[q - 1][1] += self.free.pop(q)[1]

    def view(self, off: int, nbytes: int) -> torch.Tensor:
        return self.mem[off:off + nbytes]

    def free_bytes(self) -> int:
        return sum(size for _, size in self.free)

    def close(self):
        self.mem = None
        self.free = []


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
                 budget_bytes: int = 96 << 30, device: Optional[torch.device] = None,
                 prep_group: int = 32):
        self.options = options
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.Stream(self.device)        # batch iteration
        self.side = torch.cuda.Stream(self.device)          # setup + factorization
        self.batch = Batch(capacity, max_elements, device=self.device, stream=self.stream)
        self.prep_batch = Batch(prep_group, max_elements, device=self.device, stream=self.side)
        self.prep_group = prep_group
        self.capacity = capacity
        self.budget = budget_bytes
        self.pool = WorkspacePool(budget_bytes, self.device)
        self.lock = threading.Lock()
        self.resident: "collections.OrderedDict[int, Solver]" = collections.OrderedDict()
        self.busy: Dict[int, bool] = {}                     # op_id -> member in the batch
        self.queued: Dict[int, int] = {}                    # op_id -> requests waiting in `ready`
        self.range_of: Dict[int, tuple] = {}                # op_id -> (offset, bytes) in the pool
        self._pending: Optional[tuple] = None               # range handed to the Solver being set up
        self._may_wait = True                               # _alloc may wait for memory
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
    def _alloc(self, nbytes: int):
        """A pool range of nbytes for a new operator's workspace (called by
        Solver during set-up, on the preparation thread): evicts idle
        resident operators (neither in the batch nor waiting to join it),
        least recently used first, until a range fits; while none is idle it
        waits, or raises _NoRoom when the caller may not wait."""
        if WorkspacePool.round(nbytes) > self.budget:
            raise MemoryError(f"operator workspace of {nbytes} bytes exceeds the pool ({self.budget})")
        while True:
            with self.lock:
                while True:
                    off = self.pool.take(nbytes)
                    if off is not None:
                        self._pending = (off, nbytes)
                        return self.pool.view(off, nbytes)
                    victim = next((k for k in self.resident
                                   if not self.busy.get(k, False) and not self.queued.get(k, 0)), None)
                    if victim is None:
                        break
                    self.resident.pop(victim).close()
                    self.pool.give(*self.range_of.pop(victim))
                    self.evictions += 1
            if not self._may_wait:
                raise _NoRoom()
            self.stalls += 1
            time.sleep(0.0005)

    # -- preparation thread --
    def _prep_loop(self):
        torch.cuda.set_device(self.device)
        try:
            while True:
                first = self.prep_q.get()
                if first is None:
                    return
                group = [first]
                while len(group) < self.prep_group:
                    try:
                        req = self.prep_q.get_nowait()
                    except queue.Empty:
                        break
                    if req is None:
                        self.prep_q.put(None)       # seen again after this round
                        break
                    group.append(req)
                self._prepare(group)
        except BaseException as e:      # surfaced by the main loop
            self.error = e

    def _prepare(self, group: List[Request]):
        """Queue every request of the group; operators that are not resident
        are set up and then factored together.  Only the first new operator
        of a round waits for memory; when a later one does not fit, the
        round is factored and the rest of the group starts a new round."""
        pending = list(group)
        while pending:
            new: Dict[int, Solver] = {}
            ranges: Dict[int, tuple] = {}
            later = set()                   # ids of requests for an operator set up in this round
            done = len(pending)
            try:
                for i, req in enumerate(pending):
                    with self.lock:
                        reused = req.op_id in self.resident
                        if reused:
                            self.queued[req.op_id] = self.queued.get(req.op_id, 0) + 1
                    if reused:
                        self.ready.append((req, True))
                        continue
                    if req.op_id in new:
                        later.add(id(req))
                        continue
                    self._pending = None
                    self._may_wait = not new
                    try:
                        with torch.cuda.stream(self.side):
                            solver = Solver(req.system, self.options, device=self.device,
                                            stream=self.side, workspace_alloc=self._alloc)
                    except _NoRoom:
                        done = i
                        break
                    new[req.op_id] = solver
                    ranges[req.op_id] = self._pending
                if new:
                    factor_batched(self.prep_batch, list(new.values()))
            except BaseException:
                self.side.synchronize()
                for solver in new.values():
                    solver.close()
                if self._pending is not None and self._pending not in ranges.values():
                    ranges[None] = self._pending        # a set-up that failed after its range
                with self.lock:
                    for r in ranges.values():
                        self.pool.give(*r)
                raise
            with self.lock:
                for op, solver in new.items():
                    self.resident[op] = solver
                    self.range_of[op] = ranges[op]
                for req in pending[:done]:
                    if req.op_id in new:
                        self.queued[req.op_id] = self.queued.get(req.op_id, 0) + 1
            for req in pending[:done]:
                if req.op_id in new:
                    self.ready.append((req, id(req) in later))
            pending = pending[done:]

    # -- main loop --
    def _admit_ready(self):
        skipped = collections.deque()
        while self.ready and len(self.active) < self.capacity:
            req, reused = self.ready.popleft()
            with self.lock:
                if self.busy.get(req.op_id, False):
                    skipped.append((req, reused))      # its handle is still iterating
                    continue
                solver = self.resident[req.op_id]    # queued operators are never evicted
                self.resident.move_to_end(req.op_id)
                self.busy[req.op_id] = True
                self.queued[req.op_id] -= 1
            st = self.batch.admit(solver, req.rhs, tag=req.rid)
            if st != OK:
                with self.lock:
                    self.busy[req.op_id] = False
                    self.queued[req.op_id] += 1
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

    def run(self, requests: List[Request], progress=None, every: float = 10.0) -> List[Result]:
        """Replay requests at their arrival times until all have completed;
        progress(done, total), if given, is called every `every` seconds."""
        torch.cuda.synchronize(self.device)     # right-hand sides written on other streams
        self.t0 = time.perf_counter()
        pending = sorted(requests, key=lambda r: r.arrival)
        k = 0
        next_report = every
        while k < len(pending) or len(self.results) < len(pending):
            now = time.perf_counter() - self.t0
            if progress is not None and now >= next_report:
                progress(len(self.results), len(pending))
                next_report = now + every
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
        self.prep_batch.close()
        for s in self.resident.values():
            s.close()
        self.resident.clear()
        self.range_of.clear()
        self.pool.close()


def latency_stats(results: List[Result]) -> dict:
    lat = np.array([r.done - r.arrival for r in results])
    span = max(r.done for r in results) - min(r.arrival for r in results)
    return {"n": len(results), "solves_per_s": len(results) / span if span > 0 else float("nan"),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_iters": float(np.mean([r.info["iters"] for r in results])),
            "converged": int(sum(r.info["converged"] for r in results)),
            "reused": int(sum(r.reused for r in results))}

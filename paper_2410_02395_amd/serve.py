"""Continuous-batching scheduler for streams of Helmholtz solves of mixed sizes.

Requests (grid, vacuum wavenumber, medium, source, tolerance) are admitted into
*slots* of per-shape plans.  All slots of one plan iterate together: every
graph launch runs ``check_every`` iterations of Eq. 6 for each occupied slot,
and a slot whose device-side stop test has fired skips its work.  Between
launches the scheduler collects finished slots and refills them from the queue,
so new requests join while others are mid-solve.  Plans of different shapes
run on their own HIP streams and overlap on the device.  A plan is created only
while the sum of the plans' device bytes (``mbs_plan_bytes``) fits the HBM
budget; requests that do not fit wait in the queue.

Every slot's arithmetic touches only that slot's buffers and its residual
reduction has a fixed order, so a result is bitwise the same alone or in a mix.
"""

from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import Callable, Dict, List, Optional, Tuple

import torch

from . import mbs


@dataclasses.dataclass
class Request:
    """One solve: inputs already on the device; ``arrival`` in seconds from the start."""
    id: int
    arrival: float
    shape: Tuple[int, int, int]
    k0: float
    n: torch.Tensor
    S: torch.Tensor
    ramp_width: Tuple[int, int, int] = (0, 0, 0)
    ramp_max: float = 0.0
    tol: float = 1e-4
    max_iter: int = 20000
    out: Optional[torch.Tensor] = None
    admitted: Optional[float] = None
    done: Optional[float] = None
    result: Optional[dict] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class _Pool:
    def __init__(self, shape, slots, check_every, stream):
        self.shape = shape
        self.stream = stream
        self.plan = mbs.Plan(shape, (1, 1, 1), (1, 1, 1), 8, slots, 0.75, 0, check_every, stream=stream)
        self.free: List[int] = list(range(slots))
        self.busy: Dict[int, Request] = {}
        self.queue: deque = deque()


def default_slots(shape) -> int:
    vox = shape[0] * shape[1] * shape[2]
    if vox <= 128 ** 3:
        return 8
    if vox <= 192 ** 3:
        return 6
    return 4


class Server:
    """Admission, batching and completion of solve requests on one GPU."""

    def __init__(self, hbm_budget: float = 200e9, slots_for: Callable = default_slots,
                 check_every: int = 16):
        self.budget = float(hbm_budget)
        self.slots_for = slots_for
        self.check_every = int(check_every)
        self.pools: Dict[Tuple[int, int, int], _Pool] = {}
        self.used = 0
        self.pending: deque = deque()
        self.finished: List[Request] = []

    def plan_bytes(self, shape) -> int:
        return mbs.plan_bytes(shape, max_batch=self.slots_for(shape), check_every=self.check_every)

    def submit(self, req: Request):
        self.pending.append(req)

    def _evict_idle(self, need: int, keep) -> None:
        """Destroy plans with no running slot until ``need`` bytes fit the budget."""
        for shape in list(self.pools):
            if self.used + need <= self.budget:
                return
            p = self.pools[shape]
            if p.busy or shape == keep:
                continue
            p.plan.close()
            self.used -= self.plan_bytes(shape)
            del self.pools[shape]

    def _pool(self, shape) -> Optional[_Pool]:
        p = self.pools.get(shape)
        if p is not None:
            return p
        need = self.plan_bytes(shape)
        if self.used + need > self.budget:
            self._evict_idle(need, shape)
        if self.used + need > self.budget:
            return None
        p = _Pool(shape, self.slots_for(shape), self.check_every, torch.cuda.Stream())
        self.pools[shape] = p
        self.used += need
        return p

    def _admit(self, now: float):
        waiting = deque()
        while self.pending:
            r = self.pending.popleft()
            if self.plan_bytes(r.shape) > self.budget:
                # can never fit: reject instead of waiting forever
                r.admitted = r.done = now
                r.result = {"status": mbs.MBS_ENOMEM, "converged": 0, "iterations": 0}
                self.finished.append(r)
                continue
            pool = self._pool(r.shape)
            if pool is None or not pool.free:
                waiting.append(r)
                continue
            slot = pool.free.pop()
            with torch.cuda.stream(pool.stream):
                if r.out is None:
                    r.out = torch.empty(r.shape, dtype=torch.complex64, device=r.S.device)
            pool.plan.set_medium(slot, r.n, r.k0, r.ramp_width, r.ramp_max)
            pool.plan.solve_async(slot, r.S, r.tol, r.max_iter, r.out)
            r.admitted = now
            pool.busy[slot] = r
        self.pending = waiting

    def _collect(self, clock: Callable[[], float]) -> int:
        n = 0
        for pool in self.pools.values():
            for slot in list(pool.busy):
                res = pool.plan.poll(slot)
                if res is None:
                    continue
                r = pool.busy.pop(slot)
                r.done = clock()
                r.result = res
                pool.free.append(slot)
                self.finished.append(r)
                n += 1
        return n

    def busy(self) -> bool:
        return bool(self.pending) or any(p.busy for p in self.pools.values())

    def run(self, requests: List[Request], realtime: bool = True, idle_sleep: float = 2e-4) -> List[Request]:
        """Replay ``requests`` by arrival time (all at t = 0 when ``realtime`` is
        False) and return them completed."""
        todo = deque(sorted(requests, key=lambda r: r.arrival))
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
        if not realtime:
            for r in todo:
                r.arrival = 0.0
        while todo or self.busy():
            now = clock()
            while todo and todo[0].arrival <= now:
                self.submit(todo.popleft())
            self._admit(now)
            if self._collect(clock) == 0 and not self.pending:
                time.sleep(idle_sleep)
        return sorted(self.finished, key=lambda r: r.id)

    def close(self):
        for p in self.pools.values():
            p.plan.close()
        self.pools.clear()


def run_serial(requests: List[Request], realtime: bool = True, check_every: int = 16) -> List[Request]:
    """Baseline: the same requests one at a time, in arrival order, through the
    blocking ``mbs_solve`` of a one-slot plan per shape (same kernels)."""
    plans: Dict[Tuple[int, int, int], mbs.Plan] = {}
    t0 = time.perf_counter()
    reqs = sorted(requests, key=lambda r: r.arrival)
    if not realtime:
        for r in reqs:
            r.arrival = 0.0
    for r in reqs:
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        plan = plans.get(r.shape)
        if plan is None:
            plan = plans[r.shape] = mbs.Plan(r.shape, (1, 1, 1), (1, 1, 1), 8, 1, 0.75, 0, check_every)
        if r.out is None:
            r.out = torch.empty(r.shape, dtype=torch.complex64, device=r.S.device)
        r.admitted = time.perf_counter() - t0
        plan.set_medium(0, r.n, r.k0, r.ramp_width, r.ramp_max)
        _, r.result = plan.solve(0, r.S, r.tol, r.max_iter, out=r.out)
        r.done = time.perf_counter() - t0
    for p in plans.values():
        p.close()
    return reqs


def summarize(reqs: List[Request]) -> dict:
    lat = sorted(r.latency for r in reqs)
    makespan = max(r.done for r in reqs) - min(r.arrival for r in reqs)

    def pct(p):
        k = min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))
        return lat[k]

    return {
        "requests": len(reqs),
        "solves_per_s": len(reqs) / makespan,
        "makespan_s": makespan,
        "p50_latency_s": pct(50),
        "p99_latency_s": pct(99),
        "converged": sum(1 for r in reqs if r.result and r.result["converged"]),
        "iterations_total": sum(r.result["iterations"] for r in reqs if r.result),
        # voxel-updates of all solves per second of makespan (how busy the stream kept the GPU)
        "voxel_updates_per_s": sum(r.shape[0] * r.shape[1] * r.shape[2] * r.result["iterations"]
                                   for r in reqs if r.result) / makespan,
    }

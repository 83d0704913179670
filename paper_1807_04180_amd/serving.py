"""Continuous-batching request loop over libddm's slot API.

Requests are Helmholtz solves of different grids, partitions, media and
frequencies, each with one or more right-hand sides.  A factorisation is
cached per problem key and kept resident while the HBM budget allows (LRU
eviction of idle factorisations); every cached handle owns `slots` RHS slots
and its own HIP stream.  Right-hand sides join free slots at DDM step
boundaries while the other slots keep iterating, and leave when they reach
their tolerance, so requests that arrive while others are on the GPU are
admitted as slots and memory free up and their steps overlap on the device.
A slot's arithmetic does not depend on the other slots: each result is the
same alone and in the mix (alone meaning the same problem on a handle with
the same number of slots, hence the same kernels).

A cache miss builds its handle (setup and factorisation, in the tuned
configuration when the plan cache holds one for its shape) on a worker
thread with its own stream: the scheduling loop keeps stepping the other
handles meanwhile, and the request's right-hand sides join once the handle
is ready.  Its HBM is reserved when the build starts.

Everything here is host-side scheduling; all numerical work runs in libddm.
"""
from __future__ import annotations

import collections
import concurrent.futures
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Tuple

import torch

from .solver import HelmholtzDDM, Problem


@dataclasses.dataclass
class Request:
    """One solve: sources f ([nrhs, nglob] complex128 on the device) for the
    problem identified by key; make_problem() builds (Problem, k2 tensor) on a
    cache miss."""
    rid: int
    key: Tuple
    make_problem: Callable[[], Tuple[Problem, torch.Tensor]]
    f: object                       # the sources, or a callable that makes them at arrival
    tol: float = 1e-6
    max_steps: int = 400
    t_arrival: float = 0.0          # seconds on the server clock
    n_rhs: Optional[int] = None     # RHS count when f is made at arrival
    keep: bool = True               # False: drop f and u once done (relres / steps stay)
    # filled by the server
    u: Optional[torch.Tensor] = None
    relres: Optional[List[float]] = None
    steps: Optional[List[int]] = None
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    cache_hit: Optional[bool] = None

    @property
    def nrhs(self) -> int:
        if self.n_rhs is not None:
            return int(self.n_rhs)
        return int(self.f.shape[0])

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.t_arrival


@dataclasses.dataclass
class _Entry:
    key: Tuple
    solver: HelmholtzDDM
    stream: torch.cuda.Stream
    bytes: int
    owner: List[Optional[Tuple[Request, int]]]
    last_used: float
    queue: collections.deque


class Server:
    """Continuous batching of DDM solves under an HBM budget."""

    def __init__(self, hbm_budget_bytes: int, slots: int = 16, poll_steps: int = 1,
                 device: str = "cuda:0", clock: Callable[[], float] = time.perf_counter,
                 plans=None, async_build: bool = True, plan_scope: str = ""):
        self.budget = int(hbm_budget_bytes)
        self.slots = int(slots)
        self.poll_steps = int(poll_steps)
        self.device = torch.device(device)
        self._clock = clock
        self._t0 = clock()
        self.plans = plans              # tuning.PlanCache or None
        self.plan_scope = plan_scope    # cache scope the plans were tuned in (tuning.scope_of)
        self.cache: "collections.OrderedDict[Tuple, _Entry]" = collections.OrderedDict()
        self.pending: Dict[Tuple, collections.deque] = collections.defaultdict(collections.deque)
        self.building: Dict[Tuple, Tuple[concurrent.futures.Future, int, float]] = {}
        self._pool = concurrent.futures.ThreadPoolExecutor(max_workers=1) if async_build else None
        self.done: List[Request] = []
        self.hits = 0
        self.misses = 0
        self.evictions = 0
        self.bytes_in_use = 0
        self.peak_bytes = 0
        self.factor_seconds = 0.0
        self.steps_enqueued = 0
        self.plans_applied = 0

    # -- clock ---------------------------------------------------------------
    def now(self) -> float:
        return self._clock() - self._t0

    # -- admission -----------------------------------------------------------
    def submit(self, req: Request):
        if callable(req.f):
            req.f = req.f()
        # a hit: the factorisation was resident when the request arrived
        req.cache_hit = req.key in self.cache
        if req.cache_hit:
            self.hits += 1
        else:
            self.misses += 1
        for q in range(req.nrhs):
            self.pending[req.key].append((req, q))
        req.u = torch.zeros_like(req.f)
        req.relres = [None] * req.nrhs
        req.steps = [0] * req.nrhs
        req._left = req.nrhs  # type: ignore[attr-defined]

    def _idle(self, e: _Entry) -> bool:
        return all(o is None for o in e.owner) and not self.pending.get(e.key)

    def _build(self, key: Tuple, problem: Problem, k2: torch.Tensor):
        """Handle for a new problem on its own stream (worker thread): setup,
        the cached plan for its shape if any, factorisation."""
        stream = torch.cuda.Stream(self.device)
        t = self._clock()
        with torch.cuda.stream(stream):
            solver = HelmholtzDDM(problem, k2, self.slots, factor=False)
            applied = False
            if self.plans is not None:
                from .tuning import apply_plan, plan_key
                plan = self.plans.get(plan_key(solver, self.slots, self.plan_scope))
                if plan is not None:
                    apply_plan(solver, plan)
                    applied = True
            if not applied:
                solver.factor()
        stream.synchronize()
        return solver, stream, self._clock() - t, applied

    def _ensure(self, key: Tuple, req: Request) -> Optional[_Entry]:
        e = self.cache.get(key)
        if e is not None:
            self.cache.move_to_end(key)
            return e
        if key in self.building:
            fut, need, _ = self.building[key]
            if not fut.done():
                return None
            del self.building[key]
            solver, stream, secs, applied = fut.result()
            return self._install(key, solver, stream, need, secs, applied)
        problem, k2 = req.make_problem()
        need = problem.memory_required(self.slots)
        if need > self.budget:
            raise ValueError("request %d needs %d bytes, more than the whole budget %d" % (req.rid, need, self.budget))
        while self.bytes_in_use + need > self.budget:
            victim = next((k for k, v in self.cache.items() if self._idle(v)), None)
            if victim is None:
                return None  # wait until slots and memory free up
            self._evict(victim)
        # reserve the memory now; the handle is built off the scheduling path
        self.bytes_in_use += need
        self.peak_bytes = max(self.peak_bytes, self.bytes_in_use)
        if self._pool is None:
            solver, stream, secs, applied = self._build(key, problem, k2)
            return self._install(key, solver, stream, need, secs, applied)
        self.building[key] = (self._pool.submit(self._build, key, problem, k2), need, self.now())
        return None

    def _install(self, key, solver, stream, need, secs, applied) -> _Entry:
        self.factor_seconds += secs
        self.plans_applied += 1 if applied else 0
        e = _Entry(key, solver, stream, need, [None] * self.slots, self.now(), self.pending[key])
        self.cache[key] = e
        return e

    def _evict(self, key: Tuple):
        e = self.cache.pop(key)
        e.stream.synchronize()
        e.solver.close()
        self.bytes_in_use -= e.bytes
        self.evictions += 1

    # -- one scheduling round ----------------------------------------------
    def _round(self):
        # admit pending right-hand sides into free slots (creating handles)
        for key in list(self.pending.keys()):
            dq = self.pending[key]
            if not dq:
                continue
            e = self._ensure(key, dq[0][0])
            if e is None:
                continue
            for slot in range(self.slots):
                if not dq:
                    break
                if e.owner[slot] is None:
                    req, q = dq.popleft()
                    e.stream.wait_stream(torch.cuda.current_stream(self.device))
                    with torch.cuda.stream(e.stream):
                        e.solver.slot_admit(slot, req.f[q])
                    e.owner[slot] = (req, q)
                    if req.t_admit is None:
                        req.t_admit = self.now()
        # enqueue steps on every busy handle (each on its own stream), then poll
        busy = [e for e in self.cache.values() if any(o is not None for o in e.owner)]
        if not busy and self.building:
            time.sleep(0.001)  # nothing to step until a handle is built
        for e in busy:
            e.solver.slots_step(self.poll_steps)
            self.steps_enqueued += self.poll_steps
        for e in busy:
            rel, steps = e.solver.slots_poll()
            e.last_used = self.now()
            for slot, own in enumerate(e.owner):
                if own is None:
                    continue
                req, q = own
                if rel[slot] >= 0 and (rel[slot] <= req.tol or steps[slot] >= req.max_steps):
                    # the solution goes straight into the request's row, on the
                    # handle's stream (ordered after the row's zero fill by the
                    # wait at admission)
                    with torch.cuda.stream(e.stream):
                        e.solver.slot_retire(slot, req.u[q])
                    req.relres[q] = rel[slot]
                    req.steps[q] = steps[slot]
                    e.owner[slot] = None
                    req._left -= 1  # type: ignore[attr-defined]
                    if req._left == 0:  # type: ignore[attr-defined]
                        req.t_done = self.now()
                        self.done.append(req)
                        if not req.keep:
                            e.stream.synchronize()
                            req.f = req.u = None
        return len(busy)

    # -- driver --------------------------------------------------------------
    def run(self, arrivals: List[Request], time_limit: float = 600.0) -> List[Request]:
        """Serve requests, each made visible at its t_arrival (server clock,
        seconds from now).  Returns the completed requests."""
        todo = sorted(arrivals, key=lambda r: r.t_arrival)
        self._t0 = self._clock()
        i = 0
        total = len(todo)
        while len(self.done) < total:
            now = self.now()
            if now > time_limit:
                break
            while i < len(todo) and todo[i].t_arrival <= now:
                self.submit(todo[i])
                i += 1
            nbusy = self._round()
            if nbusy == 0 and not any(self.pending.values()) and i < len(todo):
                wait = todo[i].t_arrival - self.now()
                if wait > 0:
                    time.sleep(min(wait, 0.01))
        return self.done

    def close(self):
        for key, (fut, need, _) in list(self.building.items()):
            solver, stream, _, _ = fut.result()
            stream.synchronize()
            solver.close()
            self.bytes_in_use -= need
        self.building.clear()
        if self._pool is not None:
            self._pool.shutdown(wait=True)
        for key in list(self.cache.keys()):
            self._evict(key)

    def stats(self) -> dict:
        lat = sorted(r.latency for r in self.done if r.latency is not None)

        def pct(p):
            if not lat:
                return None
            k = min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))
            return lat[k]
        nrhs = sum(r.nrhs for r in self.done)
        span = max((r.t_done for r in self.done), default=0.0)
        held = sum(e.solver.device_bytes()[0] for e in self.cache.values() if hasattr(e.solver, "device_bytes"))
        return {"requests": len(self.done), "rhs": nrhs, "p50_s": pct(50), "p99_s": pct(99),
                "rhs_per_s": nrhs / span if span > 0 else None, "cache_hits": self.hits, "cache_misses": self.misses,
                "cache_hit_rate": self.hits / max(self.hits + self.misses, 1), "evictions": self.evictions,
                "hbm_reserved_bytes": self.bytes_in_use, "hbm_held_bytes": held,
                "peak_hbm_bytes": self.peak_bytes, "factor_seconds": self.factor_seconds,
                "plans_applied": self.plans_applied}

"""Continuous-batching solve server over the library's batch entry points.

Requests arrive over time; each names an array geometry (Nx, Ny, b) and a
set of port excitations (one right-hand side per port).  The server

* keeps one plan per geometry (generator spectrum + Krylov workspace resident
  in HBM) and admits new plans against an HBM budget, evicting idle plans in
  least-recently-used order;
* runs one GMRES engine per plan with `slots` columns on the plan's own
  stream, so plans of different geometries overlap on the GPU;
* admits a request's columns into free slots of its plan's running engine
  as soon as slots free up, steps every engine that has work, and retires
  columns as they finish (continuous batching: the engine never drains to
  take new work);
* records per-request latency (arrival to last column finished) and
  throughput.

Every solve step runs in the library (HIP kernels); this module only moves
device pointers and host bookkeeping.
"""
from __future__ import annotations

import collections
import ctypes
import time
from dataclasses import dataclass, field

import numpy as np

from . import Plan, gen_symmetric, plan_bytes, precond_bytes
from . import _lib
from ._lib import PREC, check


@dataclass
class Request:
    id: int
    t: float                      # arrival time (s, from the start of the run)
    key: tuple                    # (Nx, Ny, b)
    V: np.ndarray                 # (R, Nt) complex128 right-hand sides
    done_cols: int = 0
    t_done: float | None = None
    X: list = field(default_factory=list)
    info: list = field(default_factory=list)

    @property
    def R(self):
        return self.V.shape[0]


class _PlanState:
    def __init__(self, plan: Plan, slots: int):
        self.plan = plan
        self.slots = slots
        self.free = list(range(slots))[::-1]
        self.busy = {}                 # slot -> (request, column, v tensor, x tensor)
        self.queue = collections.deque()   # (request, column)
        self.stepped = False           # a step is in flight (poll it with lag 1)
        self.nstep = 0                 # batch_step calls issued on this plan
        self.admit_step = [0] * slots  # first step index that includes the slot's column
        self.last_used = 0.0

    @property
    def idle(self):
        return not self.busy and not self.queue


class Server:
    def __init__(self, geometry, slots=16, mode="mixed", tol=1e-8, restart=40, hbm_budget=64 << 30,
                 device="cuda:0", inner_tol=1e-4, max_iter=2000, precond=False):
        """geometry(key) -> (Nx, Ny, b, Nr, gen, rim_re, rim_rr) for a key (Nx, Ny, b).
        precond: give every plan the block-circulant preconditioner (its
        memory counts against the budget)."""
        import torch
        self.torch = torch
        self.geometry = geometry
        self.slots, self.mode, self.tol, self.restart = slots, mode, tol, restart
        self.inner_tol, self.max_iter, self.precond = inner_tol, max_iter, precond
        self.budget = hbm_budget
        self.device = torch.device(device)
        self.plans: "collections.OrderedDict[tuple, _PlanState]" = collections.OrderedDict()
        self._needs = {}
        self.used = 0
        self.stats = dict(plans_created=0, plans_evicted=0, steps=0, plan_create_s=0.0)

    # ----------------------------------------------------------- plans
    def _need(self, key):
        """Device bytes of a geometry's plan (and preconditioner), computed once
        per geometry: the symmetry test reads every generator entry, and a
        request waiting for memory asks again on every pass of the loop."""
        need = self._needs.get(key)
        if need is None:
            Nx, Ny, b, Nr, gen = self.geometry(key)[:5]
            sym = gen_symmetric(Nx, Ny, b, gen)
            need = plan_bytes(Nx, Ny, b, Nr, "mixed", self.slots, self.restart, symmetric=sym)
            if self.precond:
                need += precond_bytes(Nx, Ny, b, Nr, "mixed", symmetric=sym)
            self._needs[key] = need
        return need

    def _get_plan(self, key, now):
        ps = self.plans.get(key)
        if ps is not None:
            self.plans.move_to_end(key)
            ps.last_used = now
            return ps
        need = self._need(key)
        while self.used + need > self.budget:
            victim = next((k for k, p in self.plans.items() if p.idle), None)
            if victim is None:
                return None              # nothing idle to evict: the request waits
            self._evict(victim)
        Nx, Ny, b, Nr, gen, rim_re, rim_rr = self.geometry(key)
        t0 = time.perf_counter()
        plan = Plan.create(Nx, Ny, b, Nr, gen, rim_re, rim_rr, prec="mixed", max_rhs=self.slots,
                           restart=self.restart, device=self.device)
        if self.precond:
            plan.precond_create()
        o = _lib.SolveOpts()
        _lib.lib().toeplitz_solve_opts_default(ctypes.byref(o))
        o.tol, o.restart, o.mode, o.inner_tol, o.max_iter = self.tol, self.restart, PREC[self.mode], \
            self.inner_tol, self.max_iter
        o.precond = 1 if self.precond else 0
        check(_lib.lib().toeplitz_batch_begin(plan._h, ctypes.byref(o)))
        self.stats["plan_create_s"] += time.perf_counter() - t0
        self.stats["plans_created"] += 1
        ps = _PlanState(plan, self.slots)
        ps.bytes = need
        ps.last_used = now
        self.plans[key] = ps
        self.used += need
        return ps

    def _evict(self, key):
        ps = self.plans.pop(key)
        check(_lib.lib().toeplitz_batch_end(ps.plan._h))
        ps.plan.close()
        del ps.plan
        self.used -= ps.bytes
        self.stats["plans_evicted"] += 1

    def warm(self, keys):
        """Create plans for these geometries ahead of time (within the budget)."""
        for k in keys:
            if self._get_plan(k, 0.0) is None:
                break

    # ------------------------------------------------------------- run
    def run(self, requests, realtime=True, max_seconds=600.0, progress=None):
        """Serve the requests (sorted by arrival).  With realtime, requests are
        admitted when the wall clock passes their arrival time; otherwise all
        are admitted as fast as slots allow (saturation).  progress(done,
        total, seconds) is called after every 64 finished requests."""
        torch = self.torch
        L = _lib.lib()
        pending = collections.deque(sorted(requests, key=lambda r: r.t))
        waiting = collections.deque()          # arrived, plan not yet admitted (HBM)
        remaining = len(pending)
        phases = (ctypes.c_int * self.slots)()
        infos = (_lib.SolveInfo * self.slots)()
        stream = torch.cuda.current_stream(self.device)
        sh = ctypes.c_void_p(stream.cuda_stream)
        t0 = time.perf_counter()
        while remaining:
            now = time.perf_counter() - t0
            if now > max_seconds:
                raise RuntimeError("serving run exceeded its time limit")
            # arrivals
            while pending and (not realtime or pending[0].t <= now):
                r = pending.popleft()
                if not realtime:
                    r.t = now
                waiting.append(r)
            # plans (HBM admission) and column queues
            still = collections.deque()
            for r in waiting:
                ps = self._get_plan(r.key, now)
                if ps is None:
                    still.append(r)
                    continue
                r.X = [None] * r.R
                r.info = [None] * r.R
                for c in range(r.R):
                    ps.queue.append((r, c))
            waiting = still
            # fill free slots
            for ps in self.plans.values():
                while ps.free and ps.queue:
                    r, c = ps.queue.popleft()
                    slot = ps.free.pop()
                    v = torch.from_numpy(r.V[c]).to(self.device)
                    x = torch.empty_like(v)
                    check(L.toeplitz_batch_admit(ps.plan._h, slot, ctypes.c_void_p(v.data_ptr()),
                                                 ctypes.c_void_p(x.data_ptr()), self.tol, 0, sh))
                    ps.busy[slot] = (r, c, v, x)
                    ps.admit_step[slot] = ps.nstep
            # step every engine with work; poll the step issued last round
            stepped = []
            for ps in self.plans.values():
                if ps.busy:
                    check(L.toeplitz_batch_step(ps.plan._h, 1))
                    ps.nstep += 1
                    self.stats["steps"] += 1
                    stepped.append(ps)
            for ps in stepped:
                if not ps.stepped:
                    ps.stepped = True
                    continue
                check(L.toeplitz_batch_poll(ps.plan._h, 1, 1, phases, infos))
                polled = ps.nstep - 2          # index of the step whose status was read
                now = time.perf_counter() - t0
                for slot in list(ps.busy):
                    # a status from before the slot's admission belongs to its previous column
                    if phases[slot] == 2 and polled >= ps.admit_step[slot]:
                        r, c, v, x = ps.busy.pop(slot)
                        i = infos[slot]
                        r.X[c] = x
                        r.info[c] = dict(iters=i.iters, outer_iters=i.outer_iters, status=i.status,
                                         relres=i.relres)
                        check(L.toeplitz_batch_release(ps.plan._h, slot))
                        ps.free.append(slot)
                        r.done_cols += 1
                        if r.done_cols == r.R:
                            r.t_done = now
                            remaining -= 1
                            if progress and (len(requests) - remaining) % 64 == 0:
                                progress(len(requests) - remaining, len(requests), now)
            for ps in self.plans.values():
                if not ps.busy:
                    ps.stepped = False
        torch.cuda.synchronize(self.device)
        wall = time.perf_counter() - t0
        return self._summary(requests, wall)

    def _summary(self, requests, wall):
        lat = np.array([r.t_done - r.t for r in requests])
        cols = sum(r.R for r in requests)
        return dict(requests=len(requests), columns=int(cols), wall_s=wall,
                    requests_per_s=len(requests) / wall, solves_per_s=cols / wall,
                    p50_ms=1e3 * float(np.percentile(lat, 50)), p99_ms=1e3 * float(np.percentile(lat, 99)),
                    max_relres=float(max(i["relres"] for r in requests for i in r.info)),
                    all_ok=all(i["status"] == 0 for r in requests for i in r.info),
                    hbm_used=self.used, **self.stats)

    def close(self):
        for k in list(self.plans):
            self._evict(k)

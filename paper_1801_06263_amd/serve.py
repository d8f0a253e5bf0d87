"""Serving loop: reconstruction requests admitted into the slots of one batch
(continuous batching) on one GPU.

A request carries a scan (geometry + spectral tables), its measured counts, a
step ratio lambda and a stopping rule (an iteration budget and/or a relative
change tolerance).  The server keeps every admitted request's sinogram, dual
and maps resident on the device, advances all of them together with
osscir_batch_iterate (one launch per stage for the whole batch, graph
replay), and between ticks of a few iterations retires the slots whose
stopping rule fired (the device stops a finished slot by itself, so a slot
never runs past its rule) and admits waiting requests, first come first
served, while a slot is free and the device memory the request needs fits
the HBM budget.  Plans are cached per scan and charged to the budget once.

The plain one-scan-at-a-time loop is the same server with one slot.  Every
request's result is bit-identical in both and whatever else is in the batch
(the batched kernels compute each slot exactly as the single-scan path).
"""
from __future__ import annotations

import collections
import dataclasses
import hashlib
import time
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    geom: object            # synth.Geometry (hashable)
    spec: object            # synth.Spectral
    counts: object          # [4, V, D] float32, host array or device tensor
    lam: float
    max_iter: int = 0       # > 0: stop after this many iterations
    tol: float = 0.0        # > 0: stop once ||f_{n+1} - f_n|| / ||f_{n+1}|| <= tol
    arrival: float = 0.0    # seconds after the start of the run
    n_inner: int = 1        # > 1: nested loops, n_inner steps per expansion point (iterations count steps)


@dataclasses.dataclass
class Result:
    rid: int
    f: object               # [3, n, n] device tensor, the final iterate
    iters: int
    rel_change: float
    arrival: float
    admitted: float
    finished: float
    failed: bool = False    # stopped because its maps stopped being finite (f holds the last iterate)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def spectral_key(spec) -> str:
    h = hashlib.sha1()
    for a in (spec.mu, spec.s, spec.n0):
        h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    return h.hexdigest()


def plan_bytes(geom) -> int:
    """Device bytes a plan holds: ray lines (32 B) and rho (4 B) per ray,
    views, the projector scratch, the back-projector's staged bins per
    (16 x 16 tile, view) (16 B) and the spectral table (small)."""
    L = geom.n_views * geom.n_bins
    np_ = geom.n + 8
    nt = (geom.n + 15) // 16
    return 36 * L + 32 * geom.n_views + 32 * np_ * np_ + 16 * nt * nt * geom.n_views + 512 * 48 * 4


def request_bytes(geom, workspace_bytes: int, n_inner: int = 1) -> int:
    """Device bytes of one admitted request: f, fbar [3][n][n], y, c [4][L]
    (FP32), the iteration workspace, and with nested loops the expansion
    point's line integrals [3][L]."""
    L = geom.n_views * geom.n_bins
    return 4 * (6 * geom.n * geom.n + 8 * L + (3 * L if n_inner > 1 else 0)) + int(workspace_bytes)


class Server:
    """Continuous batching over one osscir batch.

    backend: a callable returning (Batch, Plan class); the default is the HIP
    library's (injectable so the scheduling can be exercised without a GPU).
    """

    def __init__(self, modes, max_slots: int = 32, hbm_budget: int = 64 << 30, iters_per_tick: int = 5,
                 use_graph: bool = True, backend: Optional[Callable] = None):
        if backend is None:
            from . import Batch, Plan
            backend = (Batch, Plan)
        batch_cls, self._plan_cls = backend
        self.batch = batch_cls(modes, max_slots)
        self.max_slots = int(max_slots)
        self.hbm_budget = int(hbm_budget)
        self.iters_per_tick = int(iters_per_tick)
        self.use_graph = bool(use_graph)
        self.plans: Dict[tuple, object] = {}
        self.used = 0
        self.peak_used = 0
        self.free_slots = list(range(self.max_slots))[::-1]
        self.active: Dict[int, tuple] = {}
        self.ticks = 0

    # ------------------------------------------------------------ memory
    def _plan(self, req):
        key = (req.geom, spectral_key(req.spec))
        plan = self.plans.get(key)
        if plan is None:
            need = plan_bytes(req.geom)
            if self.used + need > self.hbm_budget:
                return None
            plan = self._plan_cls(req.geom, req.spec)
            self.plans[key] = plan
            self._charge(need)
        return plan

    def preload_plan(self, geom, spec):
        """Create (and charge) the plan of a scan ahead of its first request."""
        key = (geom, spectral_key(spec))
        if key not in self.plans:
            self.plans[key] = self._plan_cls(geom, spec)
            self._charge(plan_bytes(geom))
        return self.plans[key]

    def _charge(self, nbytes: int):
        self.used += nbytes
        self.peak_used = max(self.peak_used, self.used)

    def request_cost(self, req) -> int:
        """Bytes admitting req would add: its state and workspace, plus its
        plan if no admitted request has used that scan yet."""
        plan = self.plans.get((req.geom, spectral_key(req.spec)))
        if plan is not None:
            return request_bytes(req.geom, plan.batch_workspace_bytes, req.n_inner)
        return plan_bytes(req.geom) + request_bytes(req.geom, self._estimate_workspace(req.geom), req.n_inner)

    @staticmethod
    def _estimate_workspace(geom) -> int:
        """Upper bound of a batch slot's workspace (osscir_batch_workspace_bytes)
        before the plan exists: p and qS (12 FP32 per ray), the D_TPL partial
        sums and the packed images."""
        L = geom.n_views * geom.n_bins
        np_ = geom.n + 8
        return 48 * L + 8 * ((L + 255) // 256) + 32 * np_ * np_ + 4 * 256

    # ------------------------------------------------------------ slots
    def try_admit(self, req, now: float) -> bool:
        """Admit req into a free slot if it fits the budget."""
        if req.max_iter <= 0 and req.tol <= 0:
            raise ValueError(f"request {req.rid} has no stopping rule (max_iter or tol)")
        if not self.free_slots or self.request_cost(req) + self.used > self.hbm_budget:
            return False
        plan = self._plan(req)
        if plan is None:
            return False
        cost = request_bytes(req.geom, plan.batch_workspace_bytes, req.n_inner)
        if self.used + cost > self.hbm_budget:
            return False
        state = plan.new_state(req.counts, batch=True)
        slot = self.free_slots.pop()
        nested = {"n_inner": req.n_inner} if req.n_inner > 1 else {}
        self.batch.set_slot(slot, plan, state, req.lam, max_iter=req.max_iter, tol=req.tol, **nested)
        self._charge(cost)
        self.active[slot] = (req, state, now, cost)
        return True

    def tick(self, now_fn: Callable[[], float]) -> List[Result]:
        """Advance every running slot by iters_per_tick iterations and retire
        the slots that have stopped."""
        self.batch.iterate(self.iters_per_tick, use_graph=self.use_graph)
        status = self.batch.status()
        self.ticks += 1
        t = now_fn()
        done = []
        for slot, (req, state, t_adm, cost) in list(self.active.items()):
            st, iters, rel = status[slot]
            if st in (2, 3):  # stopped by its rule, or failed (non-finite maps)
                done.append(Result(req.rid, state.f, iters, rel, req.arrival, t_adm, t, failed=st == 3))
                self.batch.clear_slot(slot)
                del self.active[slot]
                self.free_slots.append(slot)
                self.used -= cost
        return done

    def run(self, requests: List[Request], clock: Callable[[], float] = time.perf_counter,
            sleep: Callable[[float], None] = time.sleep) -> List[Result]:
        """Serve requests arriving at their arrival times (seconds after the
        call); returns the results in completion order."""
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue: collections.deque = collections.deque()
        t0 = clock()
        now = lambda: clock() - t0  # noqa: E731
        results: List[Result] = []
        while pending or queue or self.active:
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            while queue and self.try_admit(queue[0], now()):
                queue.popleft()
            if not self.active:
                if queue:
                    raise RuntimeError(f"request {queue[0].rid} does not fit the HBM budget "
                                       f"({self.hbm_budget} bytes) even on an idle device")
                if pending:
                    sleep(max(0.0, pending[0].arrival - now()))
                continue
            results.extend(self.tick(now))
        return results

    def close(self):
        self.active.clear()
        self.batch.close()
        for p in self.plans.values():
            p.close()
        self.plans.clear()


def latency_summary(results: List[Result], makespan: float) -> dict:
    lat = np.array([r.latency for r in results])
    iters = np.array([r.iters for r in results])
    return {
        "requests": len(results),
        "failed": sum(1 for r in results if r.failed),
        "solves_per_s": round(len(results) / makespan, 4) if makespan > 0 else None,
        "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
        "p99_latency_s": round(float(np.percentile(lat, 99)), 4),
        "mean_latency_s": round(float(lat.mean()), 4),
        "makespan_s": round(makespan, 3),
        "iterations_total": int(iters.sum()),
        "iterations_per_s": round(float(iters.sum()) / makespan, 1) if makespan > 0 else None,
    }

"""Scheduling of the serving loop (admission by free slot and HBM budget,
first come first served, retirement on the device-side stopping rule),
exercised on the CPU with a stand-in batch that advances iteration counts
and a simulated clock."""
import types

import numpy as np
import pytest

import synth
from paper_1801_06263_amd.serve import Request, Server, latency_summary, plan_bytes, request_bytes


class FakePlan:
    def __init__(self, geom, spec):
        self.n, self.n_views, self.n_bins = geom.n, geom.n_views, geom.n_bins
        L = geom.n_views * geom.n_bins
        self.workspace_bytes = 48 * L + 8 * ((L + 255) // 256) + 32 * (geom.n + 8) ** 2
        self.batch_workspace_bytes = self.workspace_bytes

    def new_state(self, c, batch=False):
        return types.SimpleNamespace(f=("f", id(c)))

    def close(self):
        pass


class FakeBatch:
    """Advances each bound slot by the iterations of a tick, stopping it at
    its budget, and charges simulated time growing as the square root of the
    active slots (a batch fills the device better than one scan)."""

    def __init__(self, modes, max_slots):
        self.max_slots = max_slots
        self.slots = {}
        self.max_active = 0
        self.clock = None

    def set_slot(self, slot, plan, state, lam, max_iter=0, tol=0.0):
        assert slot not in self.slots and 0 <= slot < self.max_slots
        self.slots[slot] = [0, max_iter, lam != lam]  # a NaN step ratio stands for a slot that fails
        self.max_active = max(self.max_active, len(self.slots))

    def clear_slot(self, slot):
        del self.slots[slot]

    def iterate(self, n, use_graph=True):
        for v in self.slots.values():
            v[0] = 1 if v[2] else min(v[0] + n, v[1])
        self.clock.t += 0.001 * n * len(self.slots) ** 0.5

    def status(self):
        out = [(0, 0, 0.0)] * self.max_slots
        for s, (it, mx, bad) in self.slots.items():
            out[s] = (3 if bad and it else (2 if it >= mx else 1), it, 0.0)
        return out

    def close(self):
        pass


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


def requests(n=12, seed=0, budgets=(20, 60)):
    rng = np.random.default_rng(seed)
    spec = synth.make_spectral(20, 119, 120.0, 1e5, e_step=5)
    geoms = [synth.make_geometry(32, 20.0, 24, 48), synth.make_geometry(48, 20.0, 30, 64)]
    arr = np.cumsum(rng.exponential(0.05, n))
    return [Request(i, geoms[i % 2], spec, np.zeros((4, 1, 1), np.float32), 1e-7,
                    max_iter=int(rng.integers(*budgets)), arrival=float(arr[i])) for i in range(n)]


def serve(reqs, **kw):
    clock = SimClock()
    srv = Server(None, backend=(FakeBatch, FakePlan), **kw)
    srv.batch.clock = clock
    res = srv.run(reqs, clock=clock, sleep=clock.sleep)
    return srv, res, clock


def test_every_request_completes_at_its_budget():
    reqs = requests()
    srv, res, clock = serve(reqs, max_slots=4, iters_per_tick=5)
    assert sorted(r.rid for r in res) == [r.rid for r in reqs]
    by_id = {r.rid: r for r in reqs}
    for r in res:
        assert r.iters == by_id[r.rid].max_iter
        assert r.arrival <= r.admitted <= r.finished
    assert srv.used == sum(plan_bytes(g) for g, _ in srv.plans)
    assert not srv.active and len(srv.free_slots) == 4


def test_failed_request_is_retired_and_reported():
    """A request whose slot fails (maps no longer finite) is retired after
    the tick that saw it, flagged, and its slot and bytes are reused; the
    other requests run to their budgets."""
    import dataclasses
    reqs = requests()
    reqs[3] = dataclasses.replace(reqs[3], lam=float("nan"))
    srv, res, clock = serve(reqs, max_slots=4, iters_per_tick=5)
    assert sorted(r.rid for r in res) == [r.rid for r in reqs]
    by_id = {r.rid: r for r in reqs}
    for r in res:
        assert r.failed == (r.rid == 3)
        assert r.iters == (1 if r.failed else by_id[r.rid].max_iter)
    assert latency_summary(res, clock.t)["failed"] == 1
    assert not srv.active and len(srv.free_slots) == 4


def test_first_come_first_served():
    reqs = requests(16)
    srv, res, _ = serve(reqs, max_slots=3)
    adm = sorted(res, key=lambda r: r.rid)
    times = [r.admitted for r in adm]
    assert times == sorted(times)


def test_hbm_budget_limits_concurrency():
    reqs = requests(10)
    plans = sum(plan_bytes(g) for g in {r.geom for r in reqs})
    big = max(request_bytes(r.geom, FakePlan(r.geom, None).workspace_bytes) for r in reqs)
    budget = plans + 2 * big
    srv, res, _ = serve(reqs, max_slots=8, hbm_budget=budget)
    assert len(res) == len(reqs)
    assert srv.batch.max_active <= 2
    assert srv.peak_used <= budget


def test_one_slot_is_the_sequential_loop():
    reqs = requests(8)
    srv, res, _ = serve(reqs, max_slots=1)
    assert srv.batch.max_active == 1
    fin = [r.finished for r in sorted(res, key=lambda r: r.rid)]
    assert fin == sorted(fin)


def test_summary_under_load():
    reqs = requests(24, budgets=(40, 80))
    _, res_b, clk_b = serve(reqs, max_slots=8)
    _, res_s, clk_s = serve(reqs, max_slots=1)
    sb, ss = latency_summary(res_b, clk_b.t), latency_summary(res_s, clk_s.t)
    assert sb["requests"] == ss["requests"] == 24
    assert sb["p50_latency_s"] <= sb["p99_latency_s"] and ss["p50_latency_s"] <= ss["p99_latency_s"]
    assert sb["iterations_total"] == ss["iterations_total"] == sum(r.max_iter for r in reqs)
    assert clk_b.t < clk_s.t


def test_rejects_impossible_and_unbounded_requests():
    reqs = requests(2)
    with pytest.raises(RuntimeError):
        serve(reqs, max_slots=2, hbm_budget=1000)
    r = requests(1)[0]
    r.max_iter = 0
    with pytest.raises(ValueError):
        serve([r], max_slots=2)

"""Serving on the GPU: each request's result is the same alone and in the mix
(bit for bit: every slot of a batch computes exactly what the single-scan
path computes), under continuous batching with staggered arrivals, under an
HBM budget that limits concurrency, and in the one-slot sequential loop."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def reqs():
    """Eight requests over three scan shapes: iteration budgets and, for two,
    a relative-change tolerance; arrivals 20 ms apart."""
    from paper_1801_06263_amd import Plan
    from paper_1801_06263_amd.serve import Request
    probs = [synth.batch_slice(128, 100 + i) for i in range(4)] + [synth.batch_slice(256, 104 + i) for i in range(2)]
    tiny = synth.problem("tiny")
    probs += [tiny, tiny]
    plans = {}
    out = []
    rng = np.random.default_rng(5)
    for i, pr in enumerate(probs):
        key = pr.geom
        if key not in plans:
            plans[key] = Plan(pr.geom, pr.spec)
        plan = plans[key]
        g = pr.geom
        p = plan.forward_project(torch.as_tensor(pr.f_true.astype(np.float32)).cuda())
        chat = plan.spectral_model(p, torch.zeros(4, g.n_views, g.n_bins, device="cuda"))["chat"]
        c = synth.poisson_counts(host(chat), pr.seed + i).astype(np.float32)
        lam = 3e-7 if pr.name == "tiny" else 2e-8
        tol = 2e-3 if i in (2, 6) else 0.0
        out.append(Request(i, pr.geom, pr.spec, c, lam, max_iter=int(rng.integers(15, 40)), tol=tol,
                           arrival=0.02 * i))
    return out


def run(reqs, **kw):
    from paper_1801_06263_amd import Params
    from paper_1801_06263_amd.serve import Server
    srv = Server(Params(1.0, "block", "clip", True), **kw)
    try:
        res = srv.run(reqs)
    finally:
        ticks = srv.ticks
        srv.close()
    return {r.rid: r for r in res}, ticks


def test_same_alone_and_in_the_mix(reqs):
    mix, _ = run(reqs, max_slots=8, iters_per_tick=4)
    assert sorted(mix) == [r.rid for r in reqs]
    for r in reqs:
        alone, _ = run([r], max_slots=2, iters_per_tick=7)
        a, m = alone[r.rid], mix[r.rid]
        assert a.iters == m.iters and a.rel_change == m.rel_change
        assert torch.equal(a.f, m.f), r.rid
        assert torch.isfinite(m.f).all()
        if r.tol == 0.0:
            assert m.iters == r.max_iter
        else:
            assert m.iters <= r.max_iter and (m.rel_change <= r.tol or m.iters == r.max_iter)


def test_matches_single_scan_iterations(reqs):
    from paper_1801_06263_amd import Params, Plan
    mix, _ = run(reqs[:3], max_slots=4, iters_per_tick=5)
    for r in reqs[:3]:
        plan = Plan(r.geom, r.spec)
        st = plan.new_state(r.counts)
        plan.mocca_iterate(st, Params(r.lam, "block", "clip", True), mix[r.rid].iters)
        assert torch.equal(st.f, mix[r.rid].f)


def test_budget_and_sequential_loop_give_the_same_results(reqs):
    from paper_1801_06263_amd.serve import Server, plan_bytes, request_bytes
    mix, _ = run(reqs, max_slots=8, iters_per_tick=4)
    seq, _ = run(reqs, max_slots=1, iters_per_tick=4)
    # room for the plans and about two of the largest requests at a time
    geoms = {r.geom for r in reqs}
    big = max(request_bytes(g, Server._estimate_workspace(g)) for g in geoms)
    budget = sum(plan_bytes(g) for g in geoms) + 2 * big + 1
    tight, _ = run(reqs, max_slots=8, iters_per_tick=4, hbm_budget=budget)
    for r in reqs:
        assert torch.equal(mix[r.rid].f, seq[r.rid].f) and torch.equal(mix[r.rid].f, tight[r.rid].f), r.rid
    lat_seq = max(x.latency for x in seq.values())
    lat_mix = max(x.latency for x in mix.values())
    print(f"max latency: batched {lat_mix:.3f}s, sequential {lat_seq:.3f}s")


def test_served_request_matches_oracle(reqs):
    """A tiny-scan request with the oracle's counts, served for 100
    iterations among batch slices that arrive before and after it, against
    the FP64 oracle's MOCCA at the same iteration count."""
    import dataclasses

    from oracle import model, mocca, projector
    from paper_1801_06263_amd.serve import Request
    pr = synth.problem("tiny")
    X = projector.system_matrix(pr.geom)
    c = synth.poisson_counts(model.counts_model(X @ pr.f_true.reshape(3, -1).T, pr.spec), pr.seed)
    lam, n_it = 3e-7, 100
    ref, _ = mocca.mocca(X, c, pr.spec, lam, n_it, "block", "clip")
    g = pr.geom
    mine = Request(99, g, pr.spec, np.ascontiguousarray(c.T.reshape(4, g.n_views, g.n_bins), dtype=np.float32), lam,
                   max_iter=n_it, arrival=0.01)
    others = [dataclasses.replace(r, arrival=0.005 * i) for i, r in enumerate(reqs[:6])]
    mix, _ = run(others + [mine], max_slots=8, iters_per_tick=6)
    res = mix[99]
    assert res.iters == n_it
    f = host(res.f).reshape(3, -1)
    for m in range(3):
        rel = np.linalg.norm(f[m] - ref.f[m]) / np.linalg.norm(ref.f[m])
        print(f"served tiny request, material {m}: rel L2 vs oracle {rel:.2e}")
        assert rel <= 1e-3


def test_nested_request_served_among_single_loop_requests(reqs):
    """A tiny-scan request with four inner steps per expansion point at a
    lambda where the single loop diverges on this scan (1e-6), served among
    single-loop requests: the same bits as osscir_mocca_iterate_nested alone,
    and within 1e-3 of the oracle's nested loops."""
    import dataclasses

    from oracle import model, mocca, projector
    from paper_1801_06263_amd import Params, Plan
    from paper_1801_06263_amd.serve import Request
    pr = synth.problem("tiny")
    X = projector.system_matrix(pr.geom)
    c = synth.poisson_counts(model.counts_model(X @ pr.f_true.reshape(3, -1).T, pr.spec), pr.seed)
    lam, n_outer, n_inner = 1e-6, 10, 4
    g = pr.geom
    counts = np.ascontiguousarray(c.T.reshape(4, g.n_views, g.n_bins), dtype=np.float32)
    mine = Request(98, g, pr.spec, counts, lam, max_iter=n_outer * n_inner, arrival=0.01, n_inner=n_inner)
    others = [dataclasses.replace(r, arrival=0.005 * i) for i, r in enumerate(reqs[:5])]
    mix, _ = run(others + [mine], max_slots=8, iters_per_tick=3)
    res = mix[98]
    assert res.iters == n_outer * n_inner
    plan = Plan(g, pr.spec)
    st = plan.new_state(torch.as_tensor(counts).cuda())
    plan.mocca_iterate_nested(st, Params(lam, "block", "clip", True), n_outer, n_inner)
    torch.cuda.synchronize()
    assert torch.equal(st.f, res.f)
    ref = mocca.mocca_nested(X, c, pr.spec, lam, n_outer, n_inner, "block", "clip")
    f = host(res.f).reshape(3, -1)
    for m in range(3):
        rel = np.linalg.norm(f[m] - ref.f[m]) / np.linalg.norm(ref.f[m])
        print(f"served nested request, material {m}: rel L2 vs oracle {rel:.2e}")
        assert rel <= 1e-3

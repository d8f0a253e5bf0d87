"""GPU parity of MOCCA with nested loops (osscir_mocca_iterate_nested).

Bars: one inner step per expansion point is osscir_mocca_iterate bit for
bit; call patterns agree bit for bit; maps and duals after 25 x 4 steps
within relative L2 1e-3 of the FP64 oracle (as for the single loop), and the
final D_TPL within 1e-4 relative.  lambda = 1e-6 on the tiny workload is a
step at which the single loop diverges in the oracle (tests/test_oracle.py
shows the same on a smaller scan); only convergent runs go to the GPU.
"""
import ctypes
import warnings

import numpy as np
import pytest

import synth
from oracle import model, mocca as omocca, projector as pj

warnings.filterwarnings("ignore", category=RuntimeWarning)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def sino(a_lw, geom):
    """oracle [L, W] -> [W, V, D]"""
    return np.ascontiguousarray(a_lw.T.reshape(-1, geom.n_views, geom.n_bins))


@pytest.fixture(scope="module")
def tiny():
    from paper_1801_06263_amd import Plan
    pr = synth.problem("tiny")
    X = pj.system_matrix(pr.geom)
    c = synth.poisson_counts(model.counts_model(X @ pr.f_true.reshape(3, -1).T, pr.spec), pr.seed)
    return pr, X, c, Plan(pr.geom, pr.spec)


def same(a, b):
    torch.cuda.synchronize()
    return torch.equal(a.f, b.f) and torch.equal(a.fbar, b.fbar) and torch.equal(a.y, b.y)


@pytest.mark.parametrize("precond,curvature,fp64", [("block", "clip", True), ("diag", "window", False)])
def test_one_inner_step_is_the_single_loop(tiny, precond, curvature, fp64):
    from paper_1801_06263_amd import Params
    pr, X, c, plan = tiny
    prm = Params(3e-7, precond, curvature, fp64)
    a = plan.new_state(dev(sino(c, pr.geom)))
    b = plan.new_state(dev(sino(c, pr.geom)))
    plan.mocca_iterate(a, prm, 6)
    p0, _ = plan.mocca_iterate_nested(b, prm, 6, 1)
    assert same(a, b)
    # with D_TPL histories (every forward projection repacks fbar)
    ha = host(plan.mocca_iterate(a, prm, 3, dtpl=True))
    _, hb = plan.mocca_iterate_nested(b, prm, 3, 1, p0=p0, dtpl=True)
    assert same(a, b) and np.array_equal(ha, host(hb))


def test_call_patterns_agree_bitwise(tiny):
    from paper_1801_06263_amd import Params
    pr, X, c, plan = tiny
    prm = Params(1e-6, "block", "clip", True)

    def fresh():
        return plan.new_state(dev(sino(c, pr.geom)))

    one = fresh()
    plan.mocca_iterate_nested(one, prm, 4, 3)
    two = fresh()
    p0, _ = plan.mocca_iterate_nested(two, prm, 2, 3)
    plan.mocca_iterate_nested(two, prm, 2, 3, p0=p0)
    hist = fresh()
    _, d = plan.mocca_iterate_nested(hist, prm, 4, 3, dtpl=True)
    assert same(one, two) and same(one, hist)
    d = host(d)
    assert d.shape == (12,) and np.isfinite(d).all()
    assert d[-1] == float(plan.dtpl(hist.f, hist.c).item())
    # p0 holds X f0 of the last expansion point: fbar after nine steps
    ref = fresh()
    plan.mocca_iterate_nested(ref, prm, 3, 3)
    p = torch.empty_like(p0)
    plan.forward_project(ref.fbar, p)
    torch.cuda.synchronize()
    assert torch.equal(p, p0)


@pytest.mark.parametrize("precond,curvature,fp64", [("block", "clip", True), ("block", "window", False),
                                                    ("diag", "clip", True)])
def test_trajectory_parity(tiny, precond, curvature, fp64):
    from paper_1801_06263_amd import Params
    pr, X, c, plan = tiny
    lam, n_outer, n_inner = 1e-6, 25, 4
    if precond == "diag":
        lam = 3e-7
    ref = omocca.mocca_nested(X, c, pr.spec, lam, n_outer, n_inner, precond, curvature)
    st = plan.new_state(dev(sino(c, pr.geom)))
    _, d = plan.mocca_iterate_nested(st, Params(lam, precond, curvature, fp64), n_outer, n_inner, dtpl=True)
    f = host(st.f).reshape(3, -1)
    for m in range(3):
        rel = np.linalg.norm(f[m] - ref.f[m]) / np.linalg.norm(ref.f[m])
        print(f"{precond}/{curvature}/fp64={fp64} material {m}: rel L2 {rel:.2e}")
        assert rel <= 1e-3
    y = host(st.y).reshape(4, -1).T
    rel_y = np.linalg.norm(y - ref.y) / np.linalg.norm(ref.y)
    print(f"  dual rel L2 {rel_y:.2e}")
    assert rel_y <= 1e-3
    d_ref = model.image_objective(X, ref.f, c, pr.spec)
    assert abs(host(d)[-1] - d_ref) <= 1e-4 * d_ref


def test_argument_errors(tiny):
    from paper_1801_06263_amd import Params
    from paper_1801_06263_amd.osscir import OsscirError, _lib
    pr, X, c, plan = tiny
    prm = Params(1e-6)
    st = plan.new_state(dev(sino(c, pr.geom)))
    for n_outer, n_inner in ((1, 0), (-1, 2), (1 << 30, 4)):
        with pytest.raises(OsscirError, match="nested"):
            plan.mocca_iterate_nested(st, prm, n_outer, n_inner)
    # a NULL p0 through the C ABI
    cst = plan._c_state(st)
    cprm = prm.to_c()
    rc = _lib.osscir_mocca_iterate_nested(plan._h, ctypes.byref(cprm), ctypes.byref(cst), 1, 1, None, None, None)
    assert rc == -1
    # no outer iterations: nothing changes
    before = st.f.clone()
    plan.mocca_iterate_nested(st, prm, 0, 5)
    torch.cuda.synchronize()
    assert torch.equal(before, st.f)


def test_full_size_first_inner_step_is_the_single_loop_step():
    """At the 512^2, 720 x 1024 scan (120 energies): the first inner step of an
    outer iteration is the single-loop step bit for bit, and the inner steps
    after it are finite and move the maps."""
    from paper_1801_06263_amd import Params, Plan
    pr = synth.problem("large")
    plan = Plan(pr.geom, pr.spec)
    rng = np.random.default_rng(5)
    V, D = pr.geom.n_views, pr.geom.n_bins
    c = dev(rng.poisson(2e4, size=(4, V, D)).astype(np.float32))
    prm = Params(2e-8, "block", "clip", True)
    a, b = plan.new_state(c), plan.new_state(c)
    plan.mocca_iterate(a, prm, 1)
    p0, _ = plan.mocca_iterate_nested(b, prm, 1, 1)
    assert same(a, b)
    f1 = b.f.clone()
    plan.mocca_iterate_nested(b, prm, 1, 3, p0=p0)
    torch.cuda.synchronize()
    assert torch.isfinite(b.f).all() and torch.isfinite(b.y).all()
    assert not torch.equal(f1, b.f)


@pytest.mark.parametrize("case", ["detector", "modulated"])
def test_trajectory_parity_with_per_ray_spectral_tables(case):
    """Nested loops with one window response and incident count per detector
    bin (the per-bin kernels' nested variants), and with incident counts per
    ray and window on a shared response."""
    from paper_1801_06263_amd import Params, Plan
    pr = synth.problem("tiny")
    X = pj.system_matrix(pr.geom)
    if case == "detector":
        spec = synth.make_detector_spectral(pr.geom.n_bins, 20, 119, 120.0, 1e5, 77)
        oracle_spec = spec.for_rays(pr.geom.n_views)
    else:
        spec = oracle_spec = synth.modulated_spectral(pr.spec, pr.geom, seed=21)
    c = synth.poisson_counts(model.counts_model(X @ pr.f_true.reshape(3, -1).T, oracle_spec), pr.seed)
    lam, n_outer, n_inner = 1e-6, 10, 4
    ref = omocca.mocca_nested(X, c, oracle_spec, lam, n_outer, n_inner, "block", "clip")
    plan = Plan(pr.geom, spec)
    st = plan.new_state(dev(sino(c, pr.geom)))
    plan.mocca_iterate_nested(st, Params(lam, "block", "clip", True), n_outer, n_inner)
    f = host(st.f).reshape(3, -1)
    for m in range(3):
        rel = np.linalg.norm(f[m] - ref.f[m]) / np.linalg.norm(ref.f[m])
        print(f"{case} material {m}: rel L2 {rel:.2e}")
        assert rel <= 1e-3

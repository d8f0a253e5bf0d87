"""GPU parity: every entry point of the HIP library against the FP64 oracle.

Sizes: the tiny workload (64^2 image, 64 views x 128 bins, 100 energies) plus
ragged shapes that are not multiples of the tile sizes (image side 40 vs
16-pixel tiles, 100 bins vs 256-ray workgroups).  Bars:
  sinograms of non-negative maps: max |gpu - oracle| <= 1e-5 max |oracle|
  signed inputs (back-projections, signed maps): max |gpu - oracle| <=
    1e-5 max (|X| |input|), the error scale of FP32 weights in a signed sum
  adjointness <Xf, g> = <f, X^T g> (FP64 dots of FP32 results): 1e-6 relative
  spectral model (chat, r, G): 1e-5 normwise per quantity; Hessians 1e-4
  MOCCA maps after 100 iterations: relative L2 <= 1e-3 per material
"""
import math
import warnings

import numpy as np
import pytest

import synth
from helpers import micro_problem
from oracle import model, mocca as omocca, projector as pj, spc as ospc

warnings.filterwarnings("ignore", category=RuntimeWarning)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def normwise(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def plan_for(geom, spec):
    from paper_1801_06263_amd import Plan
    return Plan(geom, spec)


GEOMS = {
    "tiny": synth.problem("tiny").geom,
    "ragged": synth.make_geometry(40, 20.0, 30, 100),
    "offset": synth.Geometry(n=24, pixel_cm=0.7, n_views=17, n_bins=61, sid_cm=40.0, sdd_cm=90.0, bin_cm=0.9,
                             view0_rad=0.37, arc_rad=math.pi),
    # even n, odd n_bins: the detector-centre ray of each view at a multiple of
    # 90 degrees lies exactly on the grid line through the isocentre
    "edge16": synth.make_geometry(16, 20.0, 8, 33),
    "edge64": synth.make_geometry(64, 20.0, 64, 127),
}


@pytest.fixture(scope="module", params=sorted(GEOMS))
def scan(request):
    geom = GEOMS[request.param]
    spec = synth.make_spectral(20, 119, 120.0, 1e5, e_step=5)
    X = pj.system_matrix(geom)
    return request.param, geom, spec, X, plan_for(geom, spec)


def test_ray_lengths_match_closed_form(scan):
    name, geom, spec, X, plan = scan
    rho = host(plan.ray_lengths()).ravel()
    ref = pj.square_chord(geom)
    assert normwise(rho, ref) <= 1e-5
    assert ((rho > 0) == (ref > 1e-4)).mean() > 0.999


def test_forward_projection_parity(scan):
    name, geom, spec, X, plan = scan
    rng = np.random.default_rng(1)
    f = rng.random((3, geom.n, geom.n)).astype(np.float32)
    p = host(plan.forward_project(dev(f)))
    ref = (X @ f.reshape(3, -1).astype(np.float64).T).T.reshape(3, geom.n_views, geom.n_bins)
    assert normwise(p, ref) <= 1e-5


def signed_bar(err, X, x):
    """max |err| / max(|X| |x|): error relative to the sum of |terms|."""
    mag = (abs(X) @ np.abs(x.reshape(x.shape[0], -1)).T).T
    return np.abs(err).max() / mag.max()


def test_back_projection_parity(scan):
    name, geom, spec, X, plan = scan
    rng = np.random.default_rng(2)
    q = rng.standard_normal((9, geom.n_views, geom.n_bins)).astype(np.float32)
    b = host(plan.back_project(dev(q)))
    ref = (X.T @ q.reshape(9, -1).astype(np.float64).T).T.reshape(9, geom.n, geom.n)
    assert signed_bar((b - ref).reshape(9, -1), X.T, q.astype(np.float64)) <= 1e-5
    # non-negative input: plain normwise bar
    qa = np.abs(q)
    ba = host(plan.back_project(dev(qa)))
    refa = (X.T @ qa.reshape(9, -1).astype(np.float64).T).T.reshape(9, geom.n, geom.n)
    assert normwise(ba, refa) <= 1e-5


@pytest.mark.parametrize("nch", [1, 2, 4, 7])
def test_projection_channel_counts(scan, nch):
    name, geom, spec, X, plan = scan
    rng = np.random.default_rng(nch)
    f = rng.random((nch, geom.n, geom.n)).astype(np.float32)
    p = host(plan.forward_project(dev(f)))
    ref = (X @ f.reshape(nch, -1).astype(np.float64).T).T.reshape(p.shape)
    assert normwise(p, ref) <= 1e-5
    q = rng.standard_normal((nch, geom.n_views, geom.n_bins)).astype(np.float32)
    b = host(plan.back_project(dev(q)))
    ref = (X.T @ q.reshape(nch, -1).astype(np.float64).T).T.reshape(b.shape)
    assert signed_bar((b - ref).reshape(nch, -1), X.T, q.astype(np.float64)) <= 1e-5


def test_adjointness(scan):
    name, geom, spec, X, plan = scan
    rng = np.random.default_rng(3)
    f = rng.standard_normal((3, geom.n, geom.n)).astype(np.float32)
    g = rng.standard_normal((3, geom.n_views, geom.n_bins)).astype(np.float32)
    xf = host(plan.forward_project(dev(f)))
    xtg = host(plan.back_project(dev(g)))
    lhs = float(np.sum(xf * g.astype(np.float64)))
    rhs = float(np.sum(f.astype(np.float64) * xtg))
    scale = float(np.sum(np.abs(xf) * np.abs(g)))
    assert abs(lhs - rhs) <= 1e-6 * scale


def test_transpose_is_exact_on_unit_vectors():
    """Weights of X and X^T are the same FP32 numbers: X e_k read through the
    forward projector equals row k of X^T e_l read through the back-projector."""
    geom = GEOMS["ragged"]
    spec = synth.make_spectral(20, 119, 120.0, 1e5, e_step=5)
    plan = plan_for(geom, spec)
    L = geom.n_views * geom.n_bins
    rng = np.random.default_rng(4)
    for k in rng.choice(geom.n * geom.n, 6, replace=False):
        e = np.zeros((1, geom.n, geom.n), np.float32); e.ravel()[k] = 1.0
        col = host(plan.forward_project(dev(e))).ravel()            # X[:, k]
        ls = np.nonzero(col)[0]
        assert ls.size > 0
        for l in ls[:: max(1, ls.size // 5)]:
            u = np.zeros((1, geom.n_views, geom.n_bins), np.float32); u.ravel()[l] = 1.0
            row = host(plan.back_project(dev(u))).ravel()           # X[l, :]
            assert row[k] == col[l]


def test_projector_is_deterministic(scan):
    name, geom, spec, X, plan = scan
    rng = np.random.default_rng(5)
    f = dev(rng.random((3, geom.n, geom.n)))
    q = dev(rng.standard_normal((9, geom.n_views, geom.n_bins)))
    a1, a2 = plan.forward_project(f), plan.forward_project(f)
    b1, b2 = plan.back_project(q), plan.back_project(q)
    assert torch.equal(a1, a2) and torch.equal(b1, b2)


# ---------------------------------------------------------------- spectral

@pytest.fixture(scope="module")
def tiny():
    pr = synth.problem("tiny")
    X = pj.system_matrix(pr.geom)
    ftrue = pr.f_true.reshape(3, -1)
    chat = model.counts_model(X @ ftrue.T, pr.spec)
    c = synth.poisson_counts(chat, pr.seed)
    plan = plan_for(pr.geom, pr.spec)
    return pr, X, c, plan


def sino(a_lw, geom):
    """oracle [L, W] -> [W, V, D]"""
    return np.ascontiguousarray(a_lw.T.reshape(-1, geom.n_views, geom.n_bins))


@pytest.mark.parametrize("fp64", [False, True])
def test_spectral_model_parity(tiny, fp64):
    pr, X, c, plan = tiny
    rng = np.random.default_rng(6)
    # over-attenuating maps (c > chat on many rays) make some Hessians indefinite
    f = pr.f_true.reshape(3, -1) * (1.3 + 0.2 * rng.standard_normal((3, X.shape[1])))
    p32 = (X @ f.T).astype(np.float32)                  # both sides read the same FP32 line integrals
    p = p32.astype(np.float64)
    out = plan.spectral_model(dev(sino(p32, pr.geom)), dev(sino(c, pr.geom)), fp64_small=fp64)
    A, B, g = model.matrices_AB(p, pr.spec)
    chat = pr.spec.n0[None, :] * g
    G = model.ray_jacobian_from_A(A, pr.spec)
    H = model.hessian_from_AB(A, B, g, c, pr.spec)
    Hp = omocca.clip_negative_curvature(H)
    assert normwise(host(out["chat"]), sino(chat, pr.geom)) <= 1e-5
    assert normwise(host(out["r"]), sino(c - chat, pr.geom)) <= 1e-5
    Gs = np.stack([G[:, w, m] for w in range(4) for m in range(3)])
    for j in range(12):
        assert normwise(host(out["G"])[j].ravel(), Gs[j]) <= 1e-5
    iu = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    Hg, Hpg = host(out["H"]).reshape(6, -1), host(out["Hplus"]).reshape(6, -1)
    for j, (m, n) in enumerate(iu):
        assert np.abs(Hg[j] - H[:, m, n]).max() <= 1e-4 * np.abs(H).max()
        assert np.abs(Hpg[j] - Hp[:, m, n]).max() <= 1e-4 * np.abs(Hp).max()
    assert (np.linalg.eigvalsh(H) < 0).any(), "test input should exercise the clip"


def test_spectral_model_zero_attenuation(tiny):
    """p = 0: chat_w = N_w exactly (window totals), G = s mu^T."""
    pr, X, c, plan = tiny
    V, D = pr.geom.n_views, pr.geom.n_bins
    out = plan.spectral_model(torch.zeros(3, V, D, device="cuda"), dev(np.zeros((4, V, D))))
    np.testing.assert_allclose(host(out["chat"]).reshape(4, -1), np.repeat(pr.spec.n0[:, None], V * D, 1), rtol=2e-6)
    G0 = pr.spec.s @ pr.spec.mu.T
    np.testing.assert_allclose(host(out["G"]).reshape(12, -1)[:, 0], G0.ravel(), rtol=2e-6)


@pytest.mark.parametrize("precond", ["block", "diag"])
def test_spc_steps_parity(tiny, precond):
    pr, X, c, plan = tiny
    p = X @ pr.f_true.reshape(3, -1).T
    G = model.ray_jacobian(p, pr.spec).astype(np.float32).astype(np.float64)
    Gd = dev(np.stack([G[:, w, m] for w in range(4) for m in range(3)]).reshape(12, pr.geom.n_views, -1))
    lam = 3e-7
    sigma, img = plan.spc_steps(Gd, lam, precond)
    rho = np.asarray(X.sum(axis=1)).ravel()
    if precond == "block":
        s_ref, tinv = ospc.block_steps_factored(G, X, rho, lam)
        iu = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
        ti = host(img).reshape(6, -1)
        for j, (m, n) in enumerate(iu):
            assert normwise(ti[j], tinv[:, m, n]) <= 1e-5
    else:
        s_ref, tau = ospc.diag_steps_factored(G, X, rho, lam)
        assert normwise(host(img).reshape(3, -1), tau.T) <= 1e-5
    # sigma * rho isolates the step formula from rho's FP32 geometry (pinned separately)
    sg = host(sigma).reshape(4, -1).T
    rho_g = host(plan.ray_lengths()).ravel()
    hit = (rho > 1e-3) & (rho_g > 0)
    np.testing.assert_allclose((sg * rho_g[:, None])[hit], (s_ref * rho[:, None])[hit], rtol=1e-5)
    assert (sg[rho_g == 0] == 0).all()


# ---------------------------------------------------------------- MOCCA

@pytest.mark.parametrize("precond,curvature,fp64", [("block", "clip", False), ("block", "clip", True),
                                                    ("block", "window", False), ("diag", "window", False)])
def test_mocca_trajectory_parity(tiny, precond, curvature, fp64):
    from paper_1801_06263_amd import Params
    pr, X, c, plan = tiny
    lam, n_it = 3e-7, 100
    ref, _ = omocca.mocca(X, c, pr.spec, lam, n_it, precond, curvature)
    st = plan.new_state(dev(sino(c, pr.geom)))
    plan.mocca_iterate(st, Params(lam, precond, curvature, fp64), n_it)
    f = host(st.f).reshape(3, -1)
    for m in range(3):
        rel = np.linalg.norm(f[m] - ref.f[m]) / np.linalg.norm(ref.f[m])
        print(f"{precond}/{curvature}/fp64={fp64} material {m}: rel L2 {rel:.2e}")
        assert rel <= 1e-3
    y = host(st.y).reshape(4, -1).T
    rel_y = np.linalg.norm(y - ref.y) / np.linalg.norm(ref.y)
    print(f"  dual rel L2 {rel_y:.2e}")
    assert rel_y <= 1e-3


def test_vector_energy_sums_trajectory_parity(tiny):
    """The spectral step with its energy sums as per-ray vector FMAs instead
    of the matrix-core contraction, on the same shared-table scan: the same
    bar against the oracle, and not the matrix-core path's bits."""
    from paper_1801_06263_amd import Params, Plan
    pr, X, c, _ = tiny
    lam, n_it = 3e-7, 100
    ref, _ = omocca.mocca(X, c, pr.spec, lam, n_it, "block", "clip")
    out = {}
    for mc in (True, False):
        plan = Plan(pr.geom, pr.spec)
        plan.set_energy_sums(mc)
        st = plan.new_state(dev(sino(c, pr.geom)))
        plan.mocca_iterate(st, Params(lam, "block", "clip", True), n_it)
        f = host(st.f).reshape(3, -1)
        for m in range(3):
            rel = np.linalg.norm(f[m] - ref.f[m]) / np.linalg.norm(ref.f[m])
            print(f"matrix_cores={mc} material {m}: rel L2 {rel:.2e}")
            assert rel <= 1e-3
        out[mc] = f
    assert not np.array_equal(out[True], out[False])


def test_energy_sums_option_is_refused_where_it_does_not_apply():
    from paper_1801_06263_amd import Plan
    from paper_1801_06263_amd.osscir import OsscirError
    geom = synth.make_geometry(16, 20.0, 8, 16)
    big = synth.make_spectral(20, 400, 420.0, 1e5)            # 381 energies: table beyond 64 KB of LDS
    plan = Plan(geom, big)
    plan.set_energy_sums(False)
    with pytest.raises(OsscirError, match="matrix cores"):
        plan.set_energy_sums(True)


def test_mu_pc_trajectory_parity(tiny):
    """mu-PC: diagonal SPC in the library's orthonormal material basis (plan
    built with mu~ = B mu, maps f = B^T g) against the oracle's mu-PC."""
    from paper_1801_06263_amd import Params, Plan
    from paper_1801_06263_amd.osscir import material_transform, mu_pc_spectral
    from oracle import mupc
    pr, X, c, plan = tiny
    lam, n_it = 1e-5, 100
    f_ref, _, _, B_ref = mupc.mocca_mu_pc(X, c, pr.spec, lam, n_it, "clip")
    spec_t, B = mu_pc_spectral(pr.spec)
    np.testing.assert_allclose(B, B_ref, rtol=1e-12, atol=1e-12 * np.abs(B_ref).max())
    plan_t = Plan(pr.geom, spec_t)
    st = plan_t.new_state(dev(sino(c, pr.geom)))
    plan_t.mocca_iterate(st, Params(lam, "diag", "clip", True), n_it)
    f = host(material_transform(B.T, st.f)).reshape(3, -1)
    for m in range(3):
        rel = np.linalg.norm(f[m] - f_ref[m]) / np.linalg.norm(f_ref[m])
        print(f"mu-PC material {m}: rel L2 {rel:.2e}")
        assert rel <= 1e-3


def test_material_transform():
    from paper_1801_06263_amd.osscir import material_transform
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 37, 37)).astype(np.float32)
    M = rng.standard_normal((3, 3))
    got = host(material_transform(M, dev(x)))
    ref = np.einsum("jm,mk->jk", M, x.reshape(3, -1).astype(np.float64)).reshape(3, 37, 37)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-6 * np.abs(ref).max())
    xd = dev(x)
    material_transform(M, xd, out=xd)  # in place
    np.testing.assert_array_equal(host(xd), got)


def test_mocca_one_step_intermediates(tiny):
    """One iteration from a non-trivial point: y and f match the oracle's parts."""
    from paper_1801_06263_amd import Params
    pr, X, c, plan = tiny
    lam = 3e-7
    rng = np.random.default_rng(9)
    f0 = (pr.f_true * (1 + 0.05 * rng.standard_normal(pr.f_true.shape))).astype(np.float32)
    parts = {}
    st0 = omocca.initial_state(3, X.shape[1], X.shape[0], 4, f0.astype(np.float64))
    omocca.mocca_step(X, np.asarray(X.sum(axis=1)).ravel(), st0, c, pr.spec, lam, "block", "clip", parts)
    st = plan.new_state(dev(sino(c, pr.geom)), dev(f0))
    plan.mocca_iterate(st, Params(lam, "block", "clip", True), 1)
    assert normwise(host(st.y).reshape(4, -1).T, parts["y"]) <= 1e-4
    df_gpu = host(st.f).reshape(3, -1) - f0.reshape(3, -1)
    df_ref = parts["f"] - f0.reshape(3, -1)
    for m in range(3):
        assert np.linalg.norm(df_gpu[m] - df_ref[m]) <= 1e-3 * np.linalg.norm(df_ref[m])


def test_mocca_one_step_negative_paths(tiny):
    """One iteration from maps with negative projections (z < 0: softexp's
    linear branch, where softexp' and softexp'' differ from softexp): y and f
    match the oracle's parts."""
    from paper_1801_06263_amd import Params
    pr, X, c, plan = tiny
    lam = 3e-7
    rng = np.random.default_rng(10)
    f0 = (-0.5 * pr.f_true * (1 + 0.05 * rng.standard_normal(pr.f_true.shape))).astype(np.float32)
    p0 = X @ f0.reshape(3, -1).T.astype(np.float64)
    assert (p0 @ pr.spec.mu < 0).mean() > 0.5  # most (ray, energy) pairs on the linear branch
    parts = {}
    st0 = omocca.initial_state(3, X.shape[1], X.shape[0], 4, f0.astype(np.float64))
    omocca.mocca_step(X, np.asarray(X.sum(axis=1)).ravel(), st0, c, pr.spec, lam, "block", "clip", parts)
    st = plan.new_state(dev(sino(c, pr.geom)), dev(f0))
    plan.mocca_iterate(st, Params(lam, "block", "clip", True), 1)
    assert normwise(host(st.y).reshape(4, -1).T, parts["y"]) <= 1e-4
    df_gpu = host(st.f).reshape(3, -1) - f0.reshape(3, -1)
    df_ref = parts["f"] - f0.reshape(3, -1)
    for m in range(3):
        assert np.linalg.norm(df_gpu[m] - df_ref[m]) <= 1e-3 * np.linalg.norm(df_ref[m])


def test_mocca_is_deterministic(tiny):
    from paper_1801_06263_amd import Params
    pr, X, c, plan = tiny
    outs = []
    for _ in range(2):
        st = plan.new_state(dev(sino(c, pr.geom)))
        plan.mocca_iterate(st, Params(3e-7, "block", "clip", False), 20)
        outs.append((st.f.clone(), st.y.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("precond", ["block", "diag"])
def test_iterate_call_patterns_agree_bitwise(tiny, precond):
    """K iterations in one call (the primal step packs fbar' for the next
    forward projection), K calls of one iteration, K x 3 stage calls, and K
    iterations with D_TPL (which repacks before every forward projection):
    identical f, fbar and y."""
    from paper_1801_06263_amd import Params
    pr, X, c, plan = tiny
    prm = Params(3e-7, precond, "clip", True)
    K = 6

    def fresh():
        return plan.new_state(dev(sino(c, pr.geom)))

    runs = []
    st = fresh()
    plan.mocca_iterate(st, prm, K)
    runs.append(st)
    st = fresh()
    for _ in range(K):
        plan.mocca_iterate(st, prm, 1)
    runs.append(st)
    st = fresh()
    for _ in range(K):
        for s in range(3):
            plan.mocca_stage(st, prm, s)
    runs.append(st)
    st = fresh()
    plan.mocca_iterate(st, prm, K, dtpl=True)
    runs.append(st)
    st = fresh()
    plan.mocca_iterate(st, prm, 2)
    plan.mocca_iterate(st, prm, K - 2)
    runs.append(st)
    torch.cuda.synchronize()
    for r in runs[1:]:
        assert torch.equal(r.f, runs[0].f) and torch.equal(r.fbar, runs[0].fbar) and torch.equal(r.y, runs[0].y)
    assert torch.isfinite(runs[0].f).all()


def test_dtpl_parity(tiny):
    from paper_1801_06263_amd import Params
    pr, X, c, plan = tiny
    f = pr.f_true.astype(np.float32)
    d = float(plan.dtpl(dev(f), dev(sino(c, pr.geom))).item())
    ref = model.image_objective(X, f.reshape(3, -1).astype(np.float64), c, pr.spec)
    assert abs(d - ref) <= 1e-4 * abs(ref)
    # D_TPL history through mocca_iterate equals separate calls
    st = plan.new_state(dev(sino(c, pr.geom)))
    hist = host(plan.mocca_iterate(st, Params(3e-7), 5, dtpl=True))
    d5 = float(plan.dtpl(st.f, st.c).item())
    assert hist[-1] == d5 and np.all(np.diff(hist) < 0)


# ---------------------------------------------------------------- per-detector-bin spectra

@pytest.fixture(scope="module")
def tiny_det():
    """The tiny scan with a calibrated-detector model: every bin its own
    window responses and incident counts (jittered thresholds, blur, gain)."""
    pr = synth.problem("tiny")
    det = synth.make_detector_spectral(pr.geom.n_bins, 20, 119, 120.0, 1e5, 77)
    rs = det.for_rays(pr.geom.n_views)
    X = pj.system_matrix(pr.geom)
    c = synth.poisson_counts(model.counts_model(X @ pr.f_true.reshape(3, -1).T, rs), pr.seed)
    return pr, det, rs, X, c, plan_for(pr.geom, det)


@pytest.mark.parametrize("fp64", [False, True])
def test_detector_spectral_model_parity(tiny_det, fp64):
    pr, det, rs, X, c, plan = tiny_det
    assert plan.per_bin
    rng = np.random.default_rng(16)
    f = pr.f_true.reshape(3, -1) * (1.3 + 0.2 * rng.standard_normal((3, X.shape[1])))
    p32 = (X @ f.T).astype(np.float32)
    p = p32.astype(np.float64)
    out = plan.spectral_model(dev(sino(p32, pr.geom)), dev(sino(c, pr.geom)), fp64_small=fp64)
    A, B, g = model.matrices_AB(p, rs)
    chat = rs.n0 * g
    G = model.ray_jacobian_from_A(A, rs)
    H = model.hessian_from_AB(A, B, g, c, rs)
    Hp = omocca.clip_negative_curvature(H)
    assert normwise(host(out["chat"]), sino(chat, pr.geom)) <= 1e-5
    assert normwise(host(out["r"]), sino(c - chat, pr.geom)) <= 1e-5
    Gs = np.stack([G[:, w, m] for w in range(4) for m in range(3)])
    for j in range(12):
        assert normwise(host(out["G"])[j].ravel(), Gs[j]) <= 1e-5
    iu = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    Hg, Hpg = host(out["H"]).reshape(6, -1), host(out["Hplus"]).reshape(6, -1)
    for j, (m, n) in enumerate(iu):
        assert np.abs(Hg[j] - H[:, m, n]).max() <= 1e-4 * np.abs(H).max()
        assert np.abs(Hpg[j] - Hp[:, m, n]).max() <= 1e-4 * np.abs(Hp).max()


def test_detector_zero_attenuation(tiny_det):
    pr, det, rs, X, c, plan = tiny_det
    V, D = pr.geom.n_views, pr.geom.n_bins
    out = plan.spectral_model(torch.zeros(3, V, D, device="cuda"), dev(np.zeros((4, V, D))))
    np.testing.assert_allclose(host(out["chat"]), sino(rs.n0, pr.geom), rtol=2e-6)


def test_detector_mocca_trajectory_and_dtpl(tiny_det):
    from paper_1801_06263_amd import Params
    pr, det, rs, X, c, plan = tiny_det
    lam, n_it = 3e-7, 100
    ref, _ = omocca.mocca(X, c, rs, lam, n_it, "block", "clip")
    st = plan.new_state(dev(sino(c, pr.geom)))
    plan.mocca_iterate(st, Params(lam, "block", "clip", True), n_it)
    f = host(st.f).reshape(3, -1)
    for m in range(3):
        rel = np.linalg.norm(f[m] - ref.f[m]) / np.linalg.norm(ref.f[m])
        print(f"detector spectra material {m}: rel L2 {rel:.2e}")
        assert rel <= 1e-3
    d = float(plan.dtpl(dev(f.reshape(3, pr.geom.n, pr.geom.n)), st.c).item())
    d_ref = model.image_objective(X, f.astype(np.float32).astype(np.float64), c, rs)
    assert abs(d - d_ref) <= 1e-4 * abs(d_ref)


def test_detector_spectra_in_a_batch(tiny_det):
    """A per-bin slot beside a shared-spectrum slot in one batch: each equals
    its single-scan run bit for bit."""
    from paper_1801_06263_amd import Batch, Params
    pr, det, rs, X, c, plan = tiny_det
    plan_s = plan_for(pr.geom, pr.spec)
    c_s = dev(sino(synth.poisson_counts(model.counts_model(X @ pr.f_true.reshape(3, -1).T, pr.spec), pr.seed),
                   pr.geom))
    c_d = dev(sino(c, pr.geom))
    b = Batch(Params(1.0, "block", "clip", True), 2)
    s0, s1 = plan.new_state(c_d), plan_s.new_state(c_s)
    b.set_slot(0, plan, s0, 3e-7)
    b.set_slot(1, plan_s, s1, 3e-7)
    b.iterate(6)
    r0, r1 = plan.new_state(c_d), plan_s.new_state(c_s)
    plan.mocca_iterate(r0, Params(3e-7, "block", "clip", True), 6)
    plan_s.mocca_iterate(r1, Params(3e-7, "block", "clip", True), 6)
    assert torch.equal(s0.f, r0.f) and torch.equal(s0.y, r0.y)
    assert torch.equal(s1.f, r1.f) and torch.equal(s1.y, r1.y)


# ---------------------------------------------------------------- per-ray incident counts

@pytest.fixture(scope="module")
def tiny_mod():
    """The tiny scan with a view-dependent tube current and a bowtie: one
    incident count per ray and window, shared window responses."""
    pr = synth.problem("tiny")
    X = pj.system_matrix(pr.geom)
    ms = synth.modulated_spectral(pr.spec, pr.geom, seed=21)
    c = synth.poisson_counts(model.counts_model(X @ pr.f_true.reshape(3, -1).T, ms), pr.seed)
    return pr, ms, X, c, plan_for(pr.geom, ms)


@pytest.mark.parametrize("fp64", [False, True])
def test_per_ray_incident_spectral_model_parity(tiny_mod, fp64):
    pr, ms, X, c, plan = tiny_mod
    rng = np.random.default_rng(17)
    f = pr.f_true.reshape(3, -1) * (1.3 + 0.2 * rng.standard_normal((3, X.shape[1])))
    p32 = (X @ f.T).astype(np.float32)
    out = plan.spectral_model(dev(sino(p32, pr.geom)), dev(sino(c, pr.geom)), fp64_small=fp64)
    p = p32.astype(np.float64)
    A, B, g = model.matrices_AB(p, ms)
    chat = ms.n0 * g
    H = model.hessian_from_AB(A, B, g, c, ms)
    assert normwise(host(out["chat"]), sino(chat, pr.geom)) <= 1e-5
    assert normwise(host(out["r"]), sino(c - chat, pr.geom)) <= 1e-5
    Hg = host(out["H"]).reshape(6, -1)
    for j, (m, n) in enumerate([(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]):
        assert np.abs(Hg[j] - H[:, m, n]).max() <= 1e-4 * np.abs(H).max()
    z = plan.spectral_model(torch.zeros(3, pr.geom.n_views, pr.geom.n_bins, device="cuda"), dev(sino(c, pr.geom)))
    np.testing.assert_allclose(host(z["chat"]), sino(ms.n0, pr.geom), rtol=2e-6)


def test_per_ray_incident_trajectory_and_dtpl(tiny_mod):
    """100 iterations (matrix-core energy sums: the response is shared) and
    D_TPL against the oracle."""
    from paper_1801_06263_amd import Params
    pr, ms, X, c, plan = tiny_mod
    lam, n_it = 3e-7, 100
    ref, _ = omocca.mocca(X, c, ms, lam, n_it, "block", "clip")
    st = plan.new_state(dev(sino(c, pr.geom)))
    plan.mocca_iterate(st, Params(lam, "block", "clip", True), n_it)
    f = host(st.f).reshape(3, -1)
    for m in range(3):
        rel = np.linalg.norm(f[m] - ref.f[m]) / np.linalg.norm(ref.f[m])
        print(f"per-ray incident counts, material {m}: rel L2 {rel:.2e}")
        assert rel <= 1e-3
    d = float(plan.dtpl(dev(f.reshape(3, pr.geom.n, pr.geom.n)), st.c).item())
    d_ref = model.image_objective(X, f.astype(np.float32).astype(np.float64), c, ms)
    assert abs(d - d_ref) <= 1e-4 * abs(d_ref)


def test_per_ray_incident_with_per_bin_responses(tiny_det):
    """Per-detector-bin responses and per-ray incident counts together."""
    pr, det, rs, X, c, _ = tiny_det
    md = synth.modulated_spectral(det, pr.geom, seed=22)
    plan = plan_for(pr.geom, md)
    assert plan.per_bin
    rr = synth.RaySpectral(mu=det.mu, s=rs.s, n0=md.n0)
    rng = np.random.default_rng(18)
    f = pr.f_true.reshape(3, -1) * (1.2 + 0.2 * rng.standard_normal((3, X.shape[1])))
    p32 = (X @ f.T).astype(np.float32)
    out = plan.spectral_model(dev(sino(p32, pr.geom)), dev(sino(c, pr.geom)), fp64_small=True)
    A, B, g = model.matrices_AB(p32.astype(np.float64), rr)
    assert normwise(host(out["chat"]), sino(md.n0 * g, pr.geom)) <= 1e-5
    G = model.ray_jacobian_from_A(A, rr)
    Gs = np.stack([G[:, w, m] for w in range(4) for m in range(3)])
    for j in range(12):
        assert normwise(host(out["G"])[j].ravel(), Gs[j]) <= 1e-5


def test_per_ray_incident_in_a_batch(tiny_mod):
    from paper_1801_06263_amd import Batch, Params
    pr, ms, X, c, plan = tiny_mod
    cd = dev(sino(c, pr.geom))
    b = Batch(Params(1.0, "block", "clip", True), 3)
    s = plan.new_state(cd)
    b.set_slot(2, plan, s, 3e-7)
    b.iterate(5)
    r = plan.new_state(cd)
    plan.mocca_iterate(r, Params(3e-7, "block", "clip", True), 5)
    assert torch.equal(s.f, r.f) and torch.equal(s.y, r.y)

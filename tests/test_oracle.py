"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every oracle function is checked here against something other than itself:
brute force, closed forms, special cases, invariants, finite differences and
the paper's one comparative claim (block-diagonal SPC converges where
diagonal SPC does not, Sec. III).  A few tests plant a mistake in a copy of
an oracle step and check that the pin catches it.
"""
import warnings

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from helpers import micro_problem, rotation
from oracle import model, mocca, projector as pj, spc

warnings.filterwarnings("ignore", category=RuntimeWarning)


# ------------------------------------------------------------ inputs (synth)

def test_attenuation_check_values():
    # mu_m(E) = a (E/30)^-3 kappa + b KN(E)/KN(30): at 30 keV exactly a + b.
    mu = synth.attenuation_table([30.0, 50.0, 51.0, 80.0])
    np.testing.assert_allclose(mu[:, 0], [0.22, 0.73, 30.9], rtol=1e-12)
    np.testing.assert_allclose(mu[:, 1:], [[0.192, 0.191, 0.174], [0.433, 0.427, 0.347],
                                           [7.326, 31.375, 8.689]], atol=1.5e-3)
    # the Gd photo-electric term jumps x5 across 50.2 keV
    e = np.array([50.0, 51.0])
    ph = mu[2, 1:3] - 0.9 * synth.klein_nishina(e) / synth.klein_nishina(30.0)
    np.testing.assert_allclose(ph[1] / ph[0], 5.0 * (50.0 / 51.0) ** 3, rtol=1e-12)


def test_spectral_response_normalised():
    sp_ = synth.make_spectral(20, 119, 120.0, 1e5)
    np.testing.assert_allclose(sp_.s.sum(axis=1), 1.0, rtol=1e-14)
    assert (sp_.s >= 0).all()
    # four overlapping windows: every adjacent pair shares energies
    for w in range(3):
        assert (np.minimum(sp_.s[w], sp_.s[w + 1]) > 1e-4).any()


# ------------------------------------------------------------ projector X

@pytest.mark.parametrize("n,views,bins,view0", [(8, 8, 16, 0.0), (12, 10, 21, 0.3)])
def test_p1_siddon_equals_bruteforce_clip(n, views, bins, view0):
    geom = synth.make_geometry(n, 20.0, views, bins)
    geom = synth.Geometry(**{**geom.__dict__, "view0_rad": view0})
    Xs = pj.system_matrix(geom).toarray()
    Xb = pj.dense_matrix_bruteforce(geom)
    np.testing.assert_allclose(Xs, Xb, atol=1e-12, rtol=0)
    assert ((Xs > 0) == (Xb > 1e-12)).all()


def test_p2_row_sums_are_square_chords():
    geom = synth.make_geometry(64, 20.0, 64, 128)
    X = pj.system_matrix(geom)
    rho = np.asarray(X.sum(axis=1)).ravel()
    ref = pj.square_chord(geom)
    np.testing.assert_allclose(rho, ref, rtol=1e-12, atol=1e-12)
    assert (ref == 0).any() and (ref > 0).mean() > 0.85    # edge bins miss the square


def test_p3_disk_chords():
    geom = synth.make_geometry(64, 20.0, 16, 64)
    X = pj.system_matrix(geom)
    cx, cy, r = 3.0, -2.0, 5.0
    disk = synth.disk_phantom(64, 20.0, [(cx, cy, r, (1.0, 0, 0))], (0.0, 0, (0, 0, 0)))[0].ravel()
    p = X @ disk
    chord, dist = pj.disk_chord(geom, cx, cy, r)
    sel = dist < r - 2 * geom.pixel_cm
    assert sel.sum() > 100
    assert np.abs(p - chord)[sel].max() < geom.pixel_cm
    # a mirrored disk (wrong sign of one axis) is far off: the pin sees flips
    wrong, _ = pj.disk_chord(geom, cx, -cy, r)
    assert np.abs(p - wrong)[sel].max() > 10 * geom.pixel_cm


def test_p4_adjoint():
    geom = synth.make_geometry(32, 20.0, 24, 48)
    X = pj.system_matrix(geom)
    rng = np.random.default_rng(4)
    f = rng.standard_normal(X.shape[1]); g = rng.standard_normal(X.shape[0])
    lhs = np.dot(X @ f, g); rhs = np.dot(f, X.T @ g)
    assert abs(lhs - rhs) <= 1e-12 * np.abs(X).sum()


def test_p5_rotation_and_mirror_symmetry():
    geom = synth.make_geometry(64, 20.0, 16, 64)
    X = pj.system_matrix(geom)
    rng = np.random.default_rng(5)
    f = rng.random((64, 64))
    p = (X @ f.ravel()).reshape(16, 64)
    # the scan rotated by a quarter turn sees the image rotated by a quarter turn
    pr = (X @ np.rot90(f, -1).ravel()).reshape(16, 64)
    np.testing.assert_allclose(np.roll(pr, -4, axis=0), p, atol=1e-11)
    # mirror y -> -y maps view beta to -beta and bin u to -u
    pm = (X @ f[::-1, :].ravel()).reshape(16, 64)
    np.testing.assert_allclose(pm[(-np.arange(16)) % 16, ::-1], p, atol=1e-11)


def test_pixel_column_matches_matrix():
    geom = synth.make_geometry(24, 20.0, 12, 40)
    X = pj.system_matrix(geom).tocsc()
    for ix, iy in [(0, 0), (5, 17), (23, 11)]:
        col = pj.pixel_column(geom, ix, iy)
        np.testing.assert_allclose(col, X[:, iy * 24 + ix].toarray().ravel(), atol=1e-12)


# ------------------------------------------------------------ counts model

def test_softexp_shape_and_cond1():
    x = np.linspace(-5, 5, 2001)
    assert np.all(model.softexp_d2(x) <= model.softexp_d1(x))          # Eq. (cond1)
    np.testing.assert_allclose(model.softexp(x[x <= 0]), np.exp(x[x <= 0]))
    np.testing.assert_allclose(model.softexp(x[x > 0]), x[x > 0] + 1)
    # value and slope continuous at 0, curvature jumps
    h = 1e-7
    assert abs(model.softexp(h) - model.softexp(-h)) < 3e-7
    assert abs(model.softexp_d1(h) - model.softexp_d1(-h)) < 3e-7
    assert model.softexp_d2(0.0) == 1.0 and model.softexp_d2(h) == 0.0


def test_p8_zero_attenuation():
    _, spec, _ = micro_problem()
    p = np.zeros((5, 3))
    chat = model.counts_model(p, spec)
    np.testing.assert_allclose(chat, np.broadcast_to(spec.n0, chat.shape), rtol=1e-15)
    A, B, g = model.matrices_AB(p, spec)
    np.testing.assert_allclose(A, np.broadcast_to(spec.s, A.shape), rtol=1e-15)
    np.testing.assert_allclose(B, A, rtol=1e-15)
    G = model.ray_jacobian(p, spec)
    np.testing.assert_allclose(G[0], spec.s @ spec.mu.T, rtol=1e-14)


def test_p8_standard_model_agrees_for_physical_paths():
    _, spec, _ = micro_problem()
    rng = np.random.default_rng(8)
    p = rng.random((50, 3)) * np.array([10.0, 1.0, 0.01])
    np.testing.assert_allclose(model.counts_model(p, spec), model.counts_model_standard(p, spec), rtol=1e-14)


def test_p9_monochromatic_beer_lambert():
    mu, length, n0 = 0.3, 2.0, 1e4
    spec = synth.Spectral(mu=np.array([[mu]]), s=np.array([[1.0]]), n0=np.array([n0]))
    X = sp.csr_matrix(np.array([[length]]))
    f_star = 1.7
    c = np.array([[n0 * np.exp(-mu * length * f_star)]])
    # the counts model is Beer-Lambert
    np.testing.assert_allclose(model.counts_model(np.array([[length * f_star]]), spec), c, rtol=1e-14)
    for pre in ("block", "diag"):
        for cur in ("clip", "window"):
            st, _ = mocca.mocca(X, c, spec, 1e-4, 300, pre, cur)
            np.testing.assert_allclose(st.f.ravel(), [np.log(n0 / c[0, 0]) / (mu * length)], rtol=1e-10)


def test_p10_gradient_by_finite_differences():
    geom, spec, f_true = micro_problem()
    X = pj.system_matrix(geom)
    c = model.counts_model(X @ f_true.reshape(3, -1).T, spec) * 1.02
    rng = np.random.default_rng(10)
    f = f_true.reshape(3, -1) * (1 + 0.05 * rng.standard_normal((3, 256)))
    f[0] += 0.05            # keep every (Zf) > 0: softexp'' jumps at 0, which spoils central differences
    grad = model.image_gradient(X, f, c, spec)
    for _ in range(3):
        d = rng.standard_normal(f.shape) * np.array([[1.0], [0.1], [0.001]])
        h = 1e-5
        fd = (model.image_objective(X, f + h * d, c, spec) - model.image_objective(X, f - h * d, c, spec)) / (2 * h)
        assert abs(fd - np.sum(grad * d)) <= 1e-7 * abs(fd) + 1e-9


def test_p10_hessian_by_finite_differences():
    _, spec, _ = micro_problem()
    rng = np.random.default_rng(11)
    p = 0.5 + rng.random((20, 3)) * np.array([10.0, 1.0, 0.01])        # z > 0 on every energy
    c = model.counts_model(p, spec) * (1 + 0.1 * rng.standard_normal((20, 4)))
    H = model.hessian_p(p, c, spec)
    for m in range(3):
        h = 1e-5 * max(1.0, abs(p[:, m]).max())
        e = np.zeros(3); e[m] = h
        fd = (model.gradient_p(p + e, c, spec) - model.gradient_p(p - e, c, spec)) / (2 * h)
        np.testing.assert_allclose(fd, H[:, :, m], rtol=1e-6, atol=1e-6 * np.abs(H).max())
    # H is symmetric and, for c > chat on some windows, indefinite in places
    np.testing.assert_allclose(H, np.swapaxes(H, 1, 2), rtol=1e-12)


def test_p10_C_nonnegative_and_A_row_sums():
    _, spec, _ = micro_problem()
    rng = np.random.default_rng(12)
    p = rng.standard_normal((200, 3)) * np.array([5.0, 1.0, 0.02])      # mixed signs: both branches
    A, B, g = model.matrices_AB(p, spec)
    assert (A - B >= 0).all()                                           # C = A - B >= 0
    assert (A.sum(axis=2) <= 1 + 1e-14).all()


def test_p14_deviance_statistics():
    from oracle import projector
    pr = synth.problem("tiny")
    X = projector.system_matrix(pr.geom)
    chat = model.counts_model(X @ pr.f_true.reshape(3, -1).T, pr.spec)
    c = synth.poisson_counts(chat, pr.seed)
    dev = 2 * model.dtpl(c, chat)
    wl = c.size
    assert abs(dev - wl) < 4 * np.sqrt(2 * wl)


# ------------------------------------------------------------ step lengths

def _random_tiny_K(seed, signed):
    rng = np.random.default_rng(seed)
    L, W, M, P = 12, 4, 3, 9
    X = rng.random((L, P)) * (rng.random((L, P)) < 0.5)
    G = rng.standard_normal((L, W, M)) if signed else rng.random((L, W, M))
    return G, X


@pytest.mark.parametrize("signed", [False, True])
def test_p6_factored_steps_equal_dense_definitions(signed):
    G, X = _random_tiny_K(6, signed)
    lam = 0.37
    K = spc.dense_K(G, X)
    rho = X.sum(axis=1)
    sig_inv_d, tinv_d = spc.block_steps_dense(K, lam, 3)
    sig_f, tinv_f = spc.block_steps_factored(G, sp.csr_matrix(X), rho, lam)
    np.testing.assert_allclose(1.0 / sig_f.T.ravel(), sig_inv_d, rtol=1e-12)
    np.testing.assert_allclose(tinv_f, tinv_d, rtol=1e-12, atol=1e-14)
    sig_d, tau_d = spc.diag_steps_dense(K, lam, 3)
    sig_f, tau_f = spc.diag_steps_factored(G, sp.csr_matrix(X), rho, lam)
    np.testing.assert_allclose(sig_f.T.ravel(), sig_d, rtol=1e-12)
    np.testing.assert_allclose(tau_f.T.ravel(), tau_d, rtol=1e-12)


def test_p6_on_model_jacobian():
    geom, spec, f_true = micro_problem(n=8, views=6, bins=12)
    X = pj.system_matrix(geom)
    p = X @ f_true.reshape(3, -1).T
    G = model.ray_jacobian(p, spec)
    rho = np.asarray(X.sum(axis=1)).ravel()
    keep = rho > 0
    K = spc.dense_K(G[keep], X.toarray()[keep])
    sig_inv_d, tinv_d = spc.block_steps_dense(K, 1e-3, 3)
    sig_f, tinv_f = spc.block_steps_factored(G[keep], X[keep], rho[keep], 1e-3)
    np.testing.assert_allclose(1.0 / sig_f.T.ravel(), sig_inv_d, rtol=1e-12)
    np.testing.assert_allclose(tinv_f, tinv_d, rtol=1e-12)


@pytest.mark.parametrize("signed", [False, True])
def test_p7_step_matrix_psd(signed):
    G, X = _random_tiny_K(7, signed)
    K = spc.dense_K(G, X)
    for lam in (0.01, 1.0, 30.0):
        sig_inv, tinv = spc.block_steps_dense(K, lam, 3)
        M = spc.assemble_M(K, tinv_blocks=tinv, sigma_inv=sig_inv)
        assert np.linalg.eigvalsh(M).min() >= -1e-12 * np.abs(M).max()
        sig, tau = spc.diag_steps_dense(K, lam, 3)
        M = spc.assemble_M(K, tau=tau, sigma=sig)
        assert np.linalg.eigvalsh(M).min() >= -1e-12 * np.abs(M).max()
    # planted mistake: dropping the 1/|K| normalisation breaks the condition
    R = K.shape[0]; P = K.shape[1] // 3
    Kr = K.reshape(R, 3, P)
    bad = np.einsum("rmk,rnk->kmn", Kr, Kr) * 0.5 / np.abs(K).max()
    M = spc.assemble_M(K, tinv_blocks=bad, sigma_inv=spc.block_steps_dense(K, 1.0, 3)[0])
    assert np.linalg.eigvalsh(M).min() < -1e-6


# ------------------------------------------------------------ curvature, prox

def test_p11_negative_curvature_clip():
    rng = np.random.default_rng(11)
    A = rng.standard_normal((50, 3, 3)); H = A + np.swapaxes(A, 1, 2)
    Hp = mocca.clip_negative_curvature(H)
    assert np.linalg.eigvalsh(Hp).min() > -1e-12
    assert np.linalg.eigvalsh(Hp - H).min() > -1e-12                # an upper bound of H
    # the nearest PSD matrix in Frobenius norm: no random PSD candidate is closer
    for _ in range(20):
        B = rng.standard_normal((50, 3, 3)); P = Hp + 0.1 * B @ np.swapaxes(B, 1, 2)
        assert (np.linalg.norm(H - P, axis=(1, 2)) >= np.linalg.norm(H - Hp, axis=(1, 2)) - 1e-12).all()
    S = A @ np.swapaxes(A, 1, 2)                                      # already PSD: unchanged
    np.testing.assert_allclose(mocca.clip_negative_curvature(S), S, atol=1e-12)
    # 2x2 block diag(a, -b) -> diag(a, 0)
    np.testing.assert_allclose(mocca.clip_negative_curvature(np.diag([2.0, -3.0, 1.0])),
                               np.diag([2.0, 0.0, 1.0]), atol=1e-15)


def test_p11_clip_curvature_reproduces_clipped_hessian():
    rng = np.random.default_rng(12)
    G = rng.standard_normal((30, 4, 3))
    A = rng.standard_normal((30, 3, 3)); H = A + np.swapaxes(A, 1, 2)
    D = mocca.curvature_clip(G, H)
    np.testing.assert_allclose(np.swapaxes(G, 1, 2) @ D @ G, mocca.clip_negative_curvature(H), atol=1e-10)
    assert np.linalg.eigvalsh(D).min() > -1e-10


def test_p11_dual_prox_optimality_and_moreau():
    rng = np.random.default_rng(13)
    L, W = 40, 4
    B = rng.standard_normal((L, W, 3)); D = B @ np.swapaxes(B, 1, 2)   # PSD rank 3
    sigma = rng.random((L, W)) + 0.1
    v, u0, r = rng.standard_normal((3, L, W))
    y = mocca.dual_prox(v, u0, sigma, r, D)
    u = (v - y) / sigma
    np.testing.assert_allclose(y, r + np.einsum("lwv,lv->lw", D, u - u0), atol=1e-12)
    # Moreau: y = v - Sigma prox_{Sigma^-1 Q}(Sigma^-1 v); the primal prox solves
    # grad Q(u) + Sigma (u - Sigma^-1 v) = 0
    lhs = D + sigma[:, :, None] * np.eye(W)[None]
    u_p = np.linalg.solve(lhs, (v - r + np.einsum("lwv,lv->lw", D, u0))[..., None])[..., 0]
    np.testing.assert_allclose(y, v - sigma * u_p, atol=1e-12)
    # window curvature with v = y_n + Sigma u0: y = (c y_n + sigma r) / (c + sigma)
    c = rng.random((L, W)) * 10 + 1
    yn = rng.standard_normal((L, W))
    yw = mocca.dual_prox(yn + sigma * u0, u0, sigma, r, mocca.curvature_window(c))
    np.testing.assert_allclose(yw, (c * yn + sigma * r) / (c + sigma), rtol=1e-12)


# ------------------------------------------------------------ MOCCA iterations

@pytest.fixture(scope="module")
def micro():
    geom, spec, f_true = micro_problem()
    X = pj.system_matrix(geom)
    c = model.counts_model(X @ f_true.reshape(3, -1).T, spec)
    return geom, spec, f_true.reshape(3, -1), X, c


@pytest.mark.parametrize("curv", ["clip", "window"])
def test_p12_block_spc_rotation_equivariant(micro, curv):
    geom, spec, f_true, X, c = micro
    R = rotation(3)
    spec_r = synth.Spectral(mu=R @ spec.mu, s=spec.s, n0=spec.n0)
    lam = 2e-7
    st, _ = mocca.mocca(X, c, spec, lam, 20, "block", curv)
    st_r, _ = mocca.mocca(X, c, spec_r, lam, 20, "block", curv)
    np.testing.assert_allclose(st_r.f, R @ st.f, rtol=0, atol=1e-9 * np.abs(st.f).max())
    # diagonal SPC is not: the paper's motivation for the block form
    sd, _ = mocca.mocca(X, c, spec, lam, 20, "diag", curv)
    sd_r, _ = mocca.mocca(X, c, spec_r, lam, 20, "diag", curv)
    assert np.abs(sd_r.f - R @ sd.f).max() > 1e-4 * np.abs(sd.f).max()


@pytest.mark.parametrize("pre", ["block", "diag"])
@pytest.mark.parametrize("curv", ["clip", "window"])
def test_p13_truth_is_a_fixed_point(micro, pre, curv):
    geom, spec, f_true, X, c = micro
    st, _ = mocca.mocca(X, c, spec, 2e-7, 5, pre, curv, f0=f_true)
    np.testing.assert_allclose(st.f, f_true, atol=1e-10)
    assert np.abs(st.y).max() < 1e-6


def test_p13_noiseless_descent(micro):
    geom, spec, f_true, X, c = micro
    d0 = model.image_objective(X, np.zeros_like(f_true), c, spec)
    st, hist = mocca.mocca(X, c, spec, 2e-7, 150, "block", "clip", dtpl_every=50)
    assert hist[-1][1] < 1e-3 * d0


def test_claim_block_spc_beats_diagonal_spc(micro):
    """Sec. III: with lambda tuned per method, block-diagonal SPC reaches a far
    lower D_TPL than diagonal SPC (which the paper reports as divergent)."""
    geom, spec, f_true, X, c = micro
    best = {}
    for pre in ("block", "diag"):
        vals = []
        for lam in (1e-7, 2e-7, 4e-7, 8e-7, 1.6e-6):
            try:
                st, hist = mocca.mocca(X, c, spec, lam, 100, pre, "clip", dtpl_every=100)
                d = hist[-1][1]
                vals.append(d if np.isfinite(d) else np.inf)
            except np.linalg.LinAlgError:
                vals.append(np.inf)
        best[pre] = min(vals)
    assert best["block"] < 0.1 * best["diag"]


# ------------------------------------------------------------ CPPD composition
#
# With the expansion point held fixed, a MOCCA step is plain CPPD (dual prox,
# primal step, extrapolation) on one fixed convex quadratic problem
# min_f Q(K f).  Written with pairs w_n = (f_{n-1}, y_n), that iteration is a
# proximal point method in the metric M = [[T^-1, -K^T], [-K, Sigma^-1]]
# (He and Yuan's reading of Chambolle-Pock), so for theta = 1 and M PSD the
# M-distance to any saddle point (f*, y*) never increases, and the iterates
# converge to the minimiser, which here has a closed form.  A dropped
# extrapolation (theta = 0, the Arrow-Hurwicz step) breaks the monotonicity.

def _composition_problem(n=8, views=12, bins=16, seed=3):
    geom = synth.make_geometry(n, 20.0, views, bins)
    spec = synth.make_spectral(20, 119, 120.0, 1e5, e_step=5)
    f_true = synth.inserts_phantom(n, 20.0)
    X = pj.system_matrix(geom)
    rho = np.asarray(X.sum(axis=1)).ravel()
    c = synth.poisson_counts(model.counts_model(X @ f_true.reshape(3, -1).T, spec), seed)
    rng = np.random.default_rng(seed)
    f0 = f_true.reshape(3, -1) * (1.0 + 0.2 * rng.standard_normal((3, n * n)))
    return spec, X, rho, c, f0


def _dense_K_from_AZ(A, mu, Xd):
    """K = A(f) Z of Sec. II as dense matrices: A [(w,l), (l',i)] is
    block-diagonal over rays, Z [(l,i), (m,k)] = mu_{m,i} X_{l,k}; rows
    w-major (w L + l), columns m-major (m P + k)."""
    L, W, I = A.shape
    M, P = mu.shape[0], Xd.shape[1]
    Ad = np.zeros((W, L, L, I))
    Ad[:, np.arange(L), np.arange(L), :] = A.transpose(1, 0, 2)
    Z = np.einsum("mi,lk->limk", mu, Xd).reshape(L * I, M * P)
    return Ad.reshape(W * L, L * I) @ Z


def _block_rows(D):
    """Per-ray W x W blocks [L, W, W] -> dense matrix in (w, l) row order."""
    L, W, _ = D.shape
    out = np.zeros((W * L, W * L))
    for l in range(L):
        idx = np.arange(W) * L + l
        out[np.ix_(idx, idx)] = D[l]
    return out


def _fixed_quadratic(spec, X, rho, c, f0, lam, precond, curv):
    """Dense K(f0), the curvature and linear term of Q, the closed-form
    minimiser f* of Q(K f) with its dual y* = grad Q(K f*), and M."""
    p0 = X @ f0.T
    A, B, g = model.matrices_AB(p0, spec)
    chat = model.incident(spec) * g
    r = model.residual(c, chat)
    G = model.ray_jacobian_from_A(A, spec)
    D = mocca.curvature_clip(G, model.hessian_from_AB(A, B, g, c, spec)) if curv == "clip" \
        else mocca.curvature_window(c)
    K = _dense_K_from_AZ(A, spec.mu, X.toarray())
    Dd = _block_rows(D)
    rr, uu = r.T.ravel(), (K @ f0.ravel())
    fs = np.linalg.solve(K.T @ Dd @ K, K.T @ (Dd @ uu - rr))
    ys = rr + Dd @ (K @ fs - uu)
    hit = np.tile(rho > 0, spec.n_win)
    ys[~hit] = 0.0
    if precond == "block":
        sinv, tinv = spc.block_steps_dense(K, lam, spec.n_mat)
        Mm = spc.assemble_M(K, tinv_blocks=tinv, sigma_inv=sinv)
    else:
        sigma, tau = spc.diag_steps_dense(K, lam, spec.n_mat)
        Mm = spc.assemble_M(K, tau=tau, sigma_inv=np.where(sigma > 0, 1.0 / np.where(sigma > 0, sigma, 1.0), 0.0))
    return K, fs, ys, Mm


def _frozen_run(spec, X, rho, c, f0, lam, precond, curv, n_it, theta, fs, ys, Mm):
    """M-distances |w_n - w*|_M^2 of the frozen-expansion iteration, w_n = (f_{n-1}, y_n)."""
    st = mocca.initial_state(3, X.shape[1], X.shape[0], spec.n_win)
    prev = st.f.copy()
    wstar = np.concatenate([fs, ys])
    dist = []
    for _ in range(n_it):
        w = np.concatenate([prev.ravel(), st.y.T.ravel()]) - wstar
        dist.append(w @ Mm @ w)
        prev = st.f.copy()
        st = mocca.mocca_step(X, rho, st, c, spec, lam, precond, curv, theta=theta, expansion=f0)
    return np.array(dist), st


@pytest.fixture(scope="module")
def composition():
    return _composition_problem()


@pytest.mark.parametrize("precond,curv,n_it", [("block", "window", 2000), ("block", "clip", 300),
                                                ("diag", "window", 300)])
def test_frozen_expansion_cppd_fejer_monotone(composition, precond, curv, n_it):
    spec, X, rho, c, f0 = composition
    lam = 1e-5
    K, fs, ys, Mm = _fixed_quadratic(spec, X, rho, c, f0, lam, precond, curv)
    # (f*, y*) is a saddle point: K^T y* = 0 and y* = grad Q(K f*)
    assert np.abs(K.T @ ys).max() <= 1e-9 * np.abs(ys).max() * np.abs(K).max()
    ev = np.linalg.eigvalsh(Mm)
    assert ev.min() >= -1e-12 * ev.max()
    dist, st = _frozen_run(spec, X, rho, c, f0, lam, precond, curv, n_it, 1.0, fs, ys, Mm)
    assert (np.diff(dist) <= 1e-10 * dist[:-1]).all()
    assert dist[-1] < 0.5 * dist[0]
    if n_it >= 2000:
        # converged to the closed-form minimiser of Q(K f)
        assert np.linalg.norm(st.f.ravel() - fs) <= 1e-5 * np.linalg.norm(fs)
        assert np.linalg.norm(st.y.T.ravel() - ys) <= 1e-3 * np.linalg.norm(ys)


@pytest.mark.parametrize("curv", ["window", "clip"])
def test_planted_no_extrapolation_breaks_fejer(composition, curv):
    # planted mistake in the oracle step: theta = 0 instead of 1
    spec, X, rho, c, f0 = composition
    lam = 1e-5
    _, fs, ys, Mm = _fixed_quadratic(spec, X, rho, c, f0, lam, "block", curv)
    dist, _ = _frozen_run(spec, X, rho, c, f0, lam, "block", curv, 100, 0.0, fs, ys, Mm)
    assert (np.diff(dist) > 1e-3 * dist[:-1]).any()


def test_nested_one_inner_step_is_mocca(composition):
    spec, X, rho, c, f0 = composition
    for precond, curv in (("block", "clip"), ("diag", "window")):
        a, _ = mocca.mocca(X, c, spec, 1e-5, 6, precond, curv, f0=f0, rho=rho)
        b = mocca.mocca_nested(X, c, spec, 1e-5, 6, 1, precond, curv, f0=f0, rho=rho)
        assert np.array_equal(a.f, b.f) and np.array_equal(a.fbar, b.fbar) and np.array_equal(a.y, b.y)


@pytest.mark.parametrize("curv", ["window", "clip"])
def test_nested_inner_loop_reaches_the_minimiser_at_its_expansion_point(composition, curv):
    # one outer iteration from f = fbar = f0: the inner steps run CPPD on
    # Q(K(f0) f) and end at its closed-form minimiser
    spec, X, rho, c, f0 = composition
    lam = 1e-5
    _, fs, _, _ = _fixed_quadratic(spec, X, rho, c, f0, lam, "block", curv)
    st = mocca.mocca_nested(X, c, spec, lam, 1, 2000, "block", curv, f0=f0, rho=rho)
    assert np.linalg.norm(st.f.ravel() - fs) <= 1e-5 * np.linalg.norm(fs)


def test_nested_outer_loop_re_expands_at_fbar(composition):
    # after a short outer iteration fbar and f differ; the next outer
    # iteration converges to the minimiser of the quadratic at fbar, not at f
    spec, X, rho, c, f0 = composition
    lam = 1e-5
    s1 = mocca.mocca_nested(X, c, spec, lam, 1, 3, "block", "window", f0=f0, rho=rho)
    _, fs_bar, _, _ = _fixed_quadratic(spec, X, rho, c, s1.fbar, lam, "block", "window")
    _, fs_f, _, _ = _fixed_quadratic(spec, X, rho, c, s1.f, lam, "block", "window")
    assert np.linalg.norm(fs_bar - fs_f) > 1e-3 * np.linalg.norm(fs_bar)
    s2 = mocca.mocca_nested(X, c, spec, lam, 1, 2000, "block", "window", rho=rho, state=s1)
    assert np.linalg.norm(s2.f.ravel() - fs_bar) <= 1e-5 * np.linalg.norm(fs_bar)
    # and two outer iterations in one call equal two calls of one
    both = mocca.mocca_nested(X, c, spec, lam, 2, 3, "block", "window", f0=f0, rho=rho)
    again = mocca.mocca_nested(X, c, spec, lam, 1, 3, "block", "window", rho=rho, state=s1)
    assert np.array_equal(both.f, again.f) and np.array_equal(both.y, again.y)


def test_nested_loops_stabilise_a_step_where_one_inner_iteration_diverges(composition):
    # Sec. III: MOCCA can diverge with a single inner iteration per expansion
    # point; at lambda = 2e-6 it does here from f = 0, while five inner
    # iterations per expansion point fit the data below the noise level
    spec, X, rho, c, _ = composition
    lam, steps = 2e-6, 200
    f_true = synth.inserts_phantom(8, 20.0).reshape(3, -1)
    floor = model.image_objective(X, f_true, c, spec)

    def final_dtpl(n_inner):
        with np.errstate(all="ignore"):
            try:
                st = mocca.mocca_nested(X, c, spec, lam, steps // n_inner, n_inner, "block", "clip", rho=rho)
            except np.linalg.LinAlgError:  # T^-1 blocks no longer invertible
                return np.inf
            d = model.image_objective(X, st.f, c, spec)
        return d if np.isfinite(d) else np.inf

    start = model.image_objective(X, np.zeros_like(f_true), c, spec)
    assert final_dtpl(1) > start
    assert final_dtpl(5) < floor


def _generic_mocca_step(spec, X, rho, c, state, lam, curv):
    """One MOCCA step from the definitions, dense: K(f0) = A(f0) Z at the
    expansion point f0 = fbar_n, Sigma and T^-1 from the paper's sums over
    K, the quadratic Q(u) = r.(u - u0) + 1/2 (u - u0)^T D (u - u0) with
    u0 = K(f0) f0, the dual prox argmin_y Q*(y) + 1/2 |y - v|^2_{Sigma^-1}
    at v = y_n + Sigma K fbar_n found by a numerical minimiser (through its
    optimality condition y = grad Q(u), u = Sigma^-1 (v - y): u minimises
    Q(u) + 1/2 u^T Sigma u - v.u), the primal step f - T K^T y with T the
    inverse of the assembled block-diagonal T^-1, and fbar = 2 f' - f."""
    from scipy.optimize import minimize
    Xd = X.toarray()
    f0 = state.fbar
    A, B, g = model.matrices_AB(Xd @ f0.T, spec)
    r = model.residual(c, model.incident(spec) * g)
    G = model.ray_jacobian_from_A(A, spec)
    D = mocca.curvature_clip(G, model.hessian_from_AB(A, B, g, c, spec)) if curv == "clip" \
        else mocca.curvature_window(c)
    K = _dense_K_from_AZ(A, spec.mu, Xd)
    sinv, tinv = spc.block_steps_dense(K, lam, spec.n_mat)
    L, W = state.y.shape
    sinv_l = sinv.reshape(W, L).T                     # [L, W]
    ray = sinv_l[:, 0] > 0                            # rays that meet the image
    u0 = (K @ f0.ravel()).reshape(W, L).T
    kfb = (K @ state.fbar.ravel()).reshape(W, L).T
    y = np.zeros((L, W))
    for l in np.flatnonzero(ray):
        sig = 1.0 / sinv_l[l]
        v = state.y[l] + sig * kfb[l]
        Dl, rl, u0l = D[l], r[l], u0[l]

        def phi(u):
            d = u - u0l
            return rl @ d + 0.5 * d @ Dl @ d + 0.5 * (sig * u) @ u - v @ u

        res = minimize(phi, np.zeros(W), jac=lambda u: rl + Dl @ (u - u0l) + sig * u - v,
                       hess=lambda u: Dl + np.diag(sig), method="trust-exact", options={"gtol": 1e-12 * np.abs(v).max()})
        y[l] = v - sig * res.x
    y = y.T.ravel()
    P = Xd.shape[1]
    Tinv = spc.assemble_M(np.zeros((0, 3 * P)), tinv_blocks=tinv, sigma_inv=np.zeros(0))
    f = state.f.ravel() - np.linalg.solve(Tinv, K.T @ y)
    fbar = 2.0 * f - state.f.ravel()
    return f.reshape(3, -1), fbar.reshape(3, -1), y.reshape(W, L).T


@pytest.mark.parametrize("curv", ["clip", "window"])
def test_mocca_step_equals_dense_cppd_definition(composition, curv):
    spec, X, rho, c, _ = composition
    lam = 1e-5
    st, _ = mocca.mocca(X, c, spec, lam, 3, "block", curv)   # a state with f != fbar and y != 0
    assert np.abs(st.f - st.fbar).max() > 1e-3 * np.abs(st.f).max()
    f_ref, fb_ref, y_ref = _generic_mocca_step(spec, X, rho, c, st, lam, curv)

    def err(s):
        return max(np.abs(s.f - f_ref).max() / np.abs(f_ref).max(),
                   np.abs(s.fbar - fb_ref).max() / np.abs(fb_ref).max(),
                   np.abs(s.y - y_ref).max() / np.abs(y_ref).max())

    assert err(mocca.mocca_step(X, rho, st, c, spec, lam, "block", curv)) <= 1e-10
    # planted mistakes in the oracle step: no extrapolation, expansion about f_n
    assert err(mocca.mocca_step(X, rho, st, c, spec, lam, "block", curv, theta=0.0)) > 1e-4
    assert err(mocca.mocca_step(X, rho, st, c, spec, lam, "block", curv, expansion="current")) > 1e-4


def test_dtpl_is_poisson_deviance_including_zero_counts():
    # Eq. (DTPL) is the Poisson log-likelihood ratio of the saturated model
    # (mean = c) over the model mean chat, summed over windows and rays; a
    # zero count contributes chat (0 log 0 = 0)
    from scipy.stats import poisson
    rng = np.random.default_rng(5)
    chat = rng.uniform(0.05, 40.0, (300, 4))
    c = rng.poisson(chat).astype(np.float64)
    c[::5, 1] = 0.0
    c[::3, 3] = 0.0
    assert (c == 0).sum() > 100
    ref = poisson.logpmf(c, c) - poisson.logpmf(c, chat)
    terms = model.dtpl_terms(c, chat)
    np.testing.assert_allclose(terms, ref, rtol=1e-10, atol=1e-12)
    np.testing.assert_array_equal(terms[c == 0], chat[c == 0])
    np.testing.assert_allclose(model.dtpl(c, chat), ref.sum(), rtol=1e-12)


# ------------------------------------------------------------ mu-PC

from oracle import mupc  # noqa: E402


def test_mupc_basis_is_weighted_gram_schmidt():
    """mu~ = B mu is orthonormal under <u, v> = sum_i w_i u_i v_i, B is lower
    triangular with a positive diagonal, and Gram-Schmidt in material order
    equals the inverse Cholesky factor of the weighted Gram matrix."""
    spec = synth.make_spectral(20, 119, 120.0, 1e5)
    B, Q = mupc.mu_pc_basis(spec)
    w = mupc.energy_weights(spec)
    assert abs(w.sum() - 1.0) < 1e-12 and (w >= 0).all()
    np.testing.assert_allclose((Q * w) @ Q.T, np.eye(3), atol=1e-12)
    np.testing.assert_allclose(Q, B @ spec.mu, atol=1e-12 * np.abs(Q).max())
    assert np.all(np.triu(B, 1) == 0) and np.all(np.diag(B) > 0)
    gram = (spec.mu * w) @ spec.mu.T
    np.testing.assert_allclose(B, np.linalg.inv(np.linalg.cholesky(gram)), atol=1e-10 * np.abs(B).max())
    # a basis orthonormalised without the spectral weights is not orthonormal under them
    _, Q_unw = mupc.mu_pc_basis(synth.Spectral(mu=spec.mu, s=np.ones_like(spec.s) / spec.s.shape[1], n0=spec.n0))
    assert np.abs((Q_unw * w) @ Q_unw.T - np.eye(3)).max() > 1e-2


def test_mupc_counts_model_is_basis_invariant(micro):
    geom, spec, f_true, X, c = micro
    spec_t, B = mupc.transformed_spectral(spec)
    rng = np.random.default_rng(7)
    g = rng.random((3, X.shape[1])) * 0.1
    f = mupc.maps_from_basis(g, B)
    np.testing.assert_allclose(model.counts_model(X @ g.T, spec_t), model.counts_model(X @ f.T, spec), rtol=1e-11)
    np.testing.assert_allclose(mupc.basis_from_maps(f, B), g, atol=1e-12)


def test_mupc_truth_is_a_fixed_point(micro):
    geom, spec, f_true, X, c = micro
    f, st, _, _ = mupc.mocca_mu_pc(X, c, spec, 1e-5, 5, "clip", f0=f_true)
    np.testing.assert_allclose(f, f_true, atol=1e-10)
    assert np.abs(st.y).max() < 1e-6


def test_claim_block_and_mupc_beat_diag(micro):
    """Sec. III, Fig. 3: with lambda tuned per method, block-diagonal SPC and
    mu-PC both end far below diagonal SPC in D_TPL.  (The paper also finds
    block SPC ahead of mu-PC; on this 16^2 problem under this reading of
    mu-PC the two are within a factor of two of each other and their order
    depends on the lambda grid, so the order is not asserted.)"""
    geom, spec, f_true, X, c = micro
    grids = {"block": (1e-7, 2e-7, 3e-7, 4e-7), "mupc": (3e-6, 6e-6, 1e-5, 1.5e-5, 2e-5),
             "diag": (1e-7, 3e-7, 1e-6)}
    best = {}
    for name, lams in grids.items():
        vals = []
        for lam in lams:
            try:
                if name == "mupc":
                    _, _, hist, _ = mupc.mocca_mu_pc(X, c, spec, lam, 100, "clip", dtpl_every=100)
                else:
                    _, hist = mocca.mocca(X, c, spec, lam, 100, name, "clip", dtpl_every=100)
                d = hist[-1][1]
                vals.append(d if np.isfinite(d) else np.inf)
            except np.linalg.LinAlgError:
                vals.append(np.inf)
        best[name] = min(vals)
    print(best)
    assert max(best["block"], best["mupc"]) < 0.1 * best["diag"]


# ------------------------------------------------------------ per-detector-bin spectra

def detector_micro(seed=21):
    geom, spec, f_true = micro_problem()
    det = synth.make_detector_spectral(geom.n_bins, 20, 119, 120.0, 1e5, seed, e_step=5)
    return geom, det, f_true


def test_detector_spectra_generator():
    _, det, _ = detector_micro()
    np.testing.assert_allclose(det.s.sum(axis=2), 1.0, rtol=1e-12)
    assert (det.s >= 0).all() and det.s.shape == (32, 4, 20)
    assert (det.n0 >= 0.5e5).all() and (det.n0 <= 1.5e5).all()
    # bins differ (jittered thresholds and gains)
    assert np.abs(det.s[0] - det.s[1]).max() > 1e-3 and np.abs(det.n0[0] - det.n0[1]).max() > 0


def test_per_ray_tables_reduce_to_shared_ones():
    """Per-ray tables that repeat the shared ones give the shared results."""
    geom, spec, f_true = micro_problem()
    X = pj.system_matrix(geom)
    L = X.shape[0]
    rs = synth.RaySpectral(mu=spec.mu, s=np.tile(spec.s, (L, 1, 1)), n0=np.tile(spec.n0, (L, 1)))
    rng = np.random.default_rng(3)
    p = X @ (f_true.reshape(3, -1) * (1 + 0.1 * rng.standard_normal((3, X.shape[1])))).T
    c = model.counts_model(p, spec) * 1.03
    np.testing.assert_allclose(model.counts_model(p, rs), model.counts_model(p, spec), rtol=1e-13)
    np.testing.assert_allclose(model.hessian_p(p, c, rs), model.hessian_p(p, c, spec), rtol=1e-11,
                               atol=1e-11 * np.abs(model.hessian_p(p, c, spec)).max())
    st_s, _ = mocca.mocca(X, c, spec, 2e-7, 5, "block", "clip")
    st_r, _ = mocca.mocca(X, c, rs, 2e-7, 5, "block", "clip")
    np.testing.assert_allclose(st_r.f, st_s.f, atol=1e-10 * np.abs(st_s.f).max())


def test_per_ray_zero_attenuation_and_monochromatic():
    geom, det, _ = detector_micro()
    rs = det.for_rays(geom.n_views)
    L = geom.n_views * geom.n_bins
    chat = model.counts_model(np.zeros((L, 3)), rs)
    np.testing.assert_allclose(chat, rs.n0, rtol=1e-15)
    # one energy per (bin, window): Beer-Lambert with that energy's attenuation
    rng = np.random.default_rng(4)
    idx = rng.integers(0, det.n_energy, (geom.n_bins, 4))
    s1 = np.zeros_like(det.s)
    for d in range(geom.n_bins):
        for w in range(4):
            s1[d, w, idx[d, w]] = 1.0
    mono = synth.DetectorSpectral(mu=det.mu, s=s1, n0=det.n0).for_rays(geom.n_views)
    p = rng.random((L, 3)) * np.array([5.0, 1.0, 0.01])
    ref = rs.n0 * np.exp(-np.einsum("lm,mlw->lw", p, det.mu[:, np.tile(idx, (geom.n_views, 1))]))
    np.testing.assert_allclose(model.counts_model(p, mono), ref, rtol=1e-13)


def test_per_ray_derivatives_by_finite_differences():
    geom, det, _ = detector_micro()
    rs = det.for_rays(geom.n_views)
    rng = np.random.default_rng(12)
    L = geom.n_views * geom.n_bins
    sub = rng.choice(L, 20, replace=False)
    rsub = synth.RaySpectral(mu=rs.mu, s=rs.s[sub], n0=rs.n0[sub])
    p = 0.5 + rng.random((20, 3)) * np.array([10.0, 1.0, 0.01])
    c = model.counts_model(p, rsub) * (1 + 0.1 * rng.standard_normal((20, 4)))
    H = model.hessian_p(p, c, rsub)
    gp = model.gradient_p(p, c, rsub)
    for m in range(3):
        h = 1e-5 * max(1.0, abs(p[:, m]).max())
        e = np.zeros(3)
        e[m] = h
        fdg = np.array([(model.dtpl(c[i], model.counts_model((p + e)[i:i + 1], _row(rsub, i))[0])
                         - model.dtpl(c[i], model.counts_model((p - e)[i:i + 1], _row(rsub, i))[0])) / (2 * h)
                        for i in range(20)])
        np.testing.assert_allclose(fdg, gp[:, m], rtol=1e-6, atol=1e-6 * np.abs(gp).max())
        fd = (model.gradient_p(p + e, c, rsub) - model.gradient_p(p - e, c, rsub)) / (2 * h)
        np.testing.assert_allclose(fd, H[:, :, m], rtol=1e-6, atol=1e-6 * np.abs(H).max())


def _row(rs, i):
    return synth.RaySpectral(mu=rs.mu, s=rs.s[i:i + 1], n0=rs.n0[i:i + 1])


def test_smoke_configuration_converges():
    """The configuration the GPU smoke check compares against (32^2, 32 views x
    64 bins, 100 energies, block SPC, clipped curvature, lambda 3e-7, 30
    iterations): the oracle's trajectory stays finite and lowers D_TPL.  On a
    5 keV energy grid (20 energies) the same run diverges, which is why the
    check uses 1 keV."""
    geom = synth.make_geometry(32, 20.0, 32, 64)
    spec = synth.make_spectral(20, 119, 120.0, 1e5)
    f_true = synth.inserts_phantom(32, 20.0)
    X = pj.system_matrix(geom)
    c = synth.poisson_counts(model.counts_model(X @ f_true.reshape(3, -1).T, spec), 7)
    st, hist = mocca.mocca(X, c, spec, 3e-7, 30, "block", "clip", dtpl_every=10)
    assert np.isfinite(st.f).all()
    d = [h[1] for h in hist]
    assert d[-1] < d[0] and d[-1] < 1e-2 * model.image_objective(X, np.zeros((3, 32 * 32)), c, spec)


def test_per_ray_incident_counts_with_a_shared_response():
    """Incident counts per ray (view-dependent) with one shared response:
    zero attenuation gives chat = N_{w,l} exactly, and every quantity equals
    the fully per-ray tables with the response repeated."""
    geom, spec, f_true = micro_problem()
    X = pj.system_matrix(geom)
    L = X.shape[0]
    ms = synth.modulated_spectral(spec, geom, seed=9)
    assert ms.n0.shape == (L, 4) and np.ptp(ms.n0[:, 0]) > 0.3 * spec.n0[0]
    np.testing.assert_allclose(model.counts_model(np.zeros((L, 3)), ms), ms.n0, rtol=1e-15)
    rs = synth.RaySpectral(mu=spec.mu, s=np.tile(spec.s, (L, 1, 1)), n0=ms.n0)
    rng = np.random.default_rng(8)
    p = X @ (f_true.reshape(3, -1) * (1 + 0.1 * rng.standard_normal((3, X.shape[1])))).T
    c = model.counts_model(p, ms) * 1.02
    np.testing.assert_allclose(model.counts_model(p, ms), model.counts_model(p, rs), rtol=1e-13)
    np.testing.assert_allclose(model.hessian_p(p, c, ms), model.hessian_p(p, c, rs), rtol=1e-11,
                               atol=1e-11 * np.abs(model.hessian_p(p, c, rs)).max())
    st_m, _ = mocca.mocca(X, c, ms, 2e-7, 5, "block", "clip")
    st_r, _ = mocca.mocca(X, c, rs, 2e-7, 5, "block", "clip")
    np.testing.assert_allclose(st_m.f, st_r.f, atol=1e-10 * np.abs(st_r.f).max())

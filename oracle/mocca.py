"""MOCCA for one-step spectral CT (Sec. I and II), FP64.

One MOCCA iteration is a CPPD step (dual prox, primal step, extrapolation
with theta = 1) on a local convex quadratic model of L_TPL around the
expansion point f0 = fbar_n, with directions of negative curvature removed,
and step lengths recomputed from K(f0) every iteration (one inner iteration
per expansion point, as in the paper's experiments).

The paper defers the exact quadratic Q to its Ref. [Barber2016b]; the reading
used here is, per ray l and with
u = (K f)_l in R^W, u0 = (K(f0) f0)_l = G_l p_l(f0):

    Q_l(u) = r_l^T (u - u0) + 1/2 (u - u0)^T D_l (u - u0)

so that grad_f Q(K f0 f) at f0 equals Z^T A^T r (the paper's gradient), with
two choices of curvature D_l:

  * "clip":   D_l = G_l^+T H_l^+ G_l^+, H_l the per-ray p-space Hessian of
              Sec. II with its negative eigenvalues set to zero (so that
              K^T D K reproduces the clipped Hessian exactly);
  * "window": D_l = diag(c_l), the PSD term Z^T A^T diag(chat + r) A Z of the
              Hessian alone.

Rays that miss the image (rho_l = 0) have a zero row in K and are masked
(y = 0).  No constraint on f is imposed (softexp removes the need), so the
primal prox is the identity.

The paper prints no iterates, so the trajectory is pinned through what the
mathematics fixes: with the expansion point held fixed the step is plain CPPD
on one convex quadratic, whose M-distance to the closed-form saddle point
never increases and whose iterates converge to the closed-form minimiser
(theta = 0 breaks it); one MOCCA step equals a dense CPPD step written from
the definitions (explicit K = A Z, the paper's sums for Sigma and T^-1, the
dual prox by a numerical minimiser); the truth is a fixed point on noiseless
data; block SPC is rotation equivariant; the monochromatic case converges to
Beer-Lambert's closed form; D_TPL descends.  The expansion point (fbar_n,
which the paper leaves unstated) is a reading; the dense cross-check holds
the oracle to it.

``mocca_nested`` runs several such fixed-quadratic steps per expansion
point; one outer iteration with many inner ones converges to the closed-form
minimiser of the quadratic at that point, and one inner step per outer
iteration is ``mocca`` bit for bit.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np

from . import model, spc


def clip_negative_curvature(H):
    """H^+ = V max(Lambda, 0) V^T for symmetric [.., M, M] (eigendecomposition)."""
    lam, V = np.linalg.eigh(H)
    return np.einsum("...ij,...j,...kj->...ik", V, np.maximum(lam, 0.0), V)


def curvature_clip(G, H):
    """D_l = G^+T H^+ G^+ with G^+ = (G^T G)^-1 G^T (Moore-Penrose, full column rank)."""
    Gp = np.linalg.pinv(G)                       # [L, M, W]
    Hp = clip_negative_curvature(H)
    return np.einsum("lmw,lmn,lnv->lwv", Gp, Hp, Gp)


def curvature_window(c):
    """D_l = diag(c_l)."""
    L, W = c.shape
    D = np.zeros((L, W, W))
    D[:, np.arange(W), np.arange(W)] = c
    return D


def dual_prox(v, u0, sigma, r, D):
    """prox of Sigma Q* at v:  argmin_y Q*(y) + 1/2 |y - v|^2_{Sigma^-1}.

    Optimality: y = grad Q(u) = r + D (u - u0) with u = Sigma^-1 (v - y), i.e.
    (I + D Sigma^-1) y = r + D (Sigma^-1 v - u0).  sigma [L, W] > 0."""
    L, W = sigma.shape
    sinv = 1.0 / sigma
    lhs = np.eye(W)[None] + D * sinv[:, None, :]
    rhs = r + np.einsum("lwv,lv->lw", D, sinv * v - u0)
    return np.linalg.solve(lhs, rhs[..., None])[..., 0]


@dataclasses.dataclass
class State:
    f: np.ndarray      # [M, P]
    fbar: np.ndarray   # [M, P]
    y: np.ndarray      # [L, W]
    n: int = 0


def initial_state(n_mat, n_pix, n_rays, n_win, f0=None) -> State:
    f = np.zeros((n_mat, n_pix)) if f0 is None else np.array(f0, dtype=np.float64).reshape(n_mat, n_pix)
    return State(f=f.copy(), fbar=f.copy(), y=np.zeros((n_rays, n_win)))


def mocca_step(X, rho, state: State, c, spec, lam: float, precond: str = "block",
               curvature: str = "clip", parts: Optional[dict] = None, theta: float = 1.0,
               expansion=None) -> State:
    """One CPPD step on the local convex quadratic of L_TPL (Sec. I, Sec. II):

        y_{n+1}    = prox_{Sigma Q*}(y_n + Sigma K(f0) fbar_n)
        f_{n+1}    = f_n - T K(f0)^T y_{n+1}
        fbar_{n+1} = f_{n+1} + theta (f_{n+1} - f_n)

    with K, Sigma, T and the quadratic Q (its r, D and u0 = K(f0) f0) formed
    at the expansion point f0.  MOCCA, one inner iteration per expansion
    point, is expansion=None (f0 = fbar_n) and theta = 1.  ``expansion`` may
    also be "current" (f0 = f_n) or a fixed [M, P] array, which turns the
    step into plain CPPD on one fixed convex quadratic.  ``parts`` (if a
    dict) receives the intermediates."""
    M = spec.n_mat
    mask = rho > 0
    pbar = X @ state.fbar.T                               # [L, M]
    if expansion is None:
        p = pbar
    elif isinstance(expansion, str):
        if expansion != "current":
            raise ValueError(expansion)
        p = X @ state.f.T
    else:
        p = X @ np.asarray(expansion, dtype=np.float64).reshape(M, -1).T
    A, B, g = model.matrices_AB(p, spec)
    chat = model.incident(spec) * g                       # Eq. (finalModel)
    r = model.residual(c, chat)
    G = model.ray_jacobian_from_A(A, spec)                # K(f0) per ray, [L, W, M]
    if curvature == "clip":
        H = model.hessian_from_AB(A, B, g, c, spec)
        D = curvature_clip(G, H)
    elif curvature == "window":
        H = None
        D = curvature_window(c)
    else:
        raise ValueError(curvature)
    if precond == "block":
        sigma, tinv = spc.block_steps_factored(G, X, rho, lam)
    elif precond == "diag":
        sigma, tau = spc.diag_steps_factored(G, X, rho, lam)
    else:
        raise ValueError(precond)
    # dual step y_{n+1} = prox_{Sigma Q*}(y_n + Sigma K(f0) fbar_n), u0 = K(f0) f0
    u0 = np.einsum("lwm,lm->lw", G, p)
    kfbar = u0 if expansion is None else np.einsum("lwm,lm->lw", G, pbar)
    y_new = np.zeros_like(state.y)
    sig_m = sigma[mask]
    y_new[mask] = dual_prox(state.y[mask] + sig_m * kfbar[mask], u0[mask], sig_m, r[mask], D[mask])
    # primal step f_{n+1} = f_n - T K^T y_{n+1}
    q = np.einsum("lwm,lw->lm", G, y_new)                 # G_l^T y_l
    b = (X.T @ q).T                                       # K^T y, [M, P]
    if precond == "block":
        f_new = state.f - np.linalg.solve(tinv, b.T[..., None])[..., 0].T
    else:
        f_new = state.f - tau.T * b
    fbar_new = f_new + theta * (f_new - state.f)
    if parts is not None:
        parts.update(p=p, chat=chat, r=r, G=G, H=H, D=D, sigma=sigma, u0=u0, y=y_new, q=q, b=b,
                     f=f_new, fbar=fbar_new)
        if precond == "block":
            parts["tinv"] = tinv
            parts["S"] = spc.ray_block_terms(G)[1]
        else:
            parts["tau"] = tau
    return State(f=f_new, fbar=fbar_new, y=y_new, n=state.n + 1)


def mocca(X, c, spec, lam: float, n_iter: int, precond: str = "block", curvature: str = "clip",
          f0=None, rho=None, dtpl_every: int = 0,
          callback: Optional[Callable[[int, State], None]] = None):
    """Run ``n_iter`` MOCCA iterations from f0 (default 0), y0 = 0.

    Returns (state, history) with history rows (n, D_TPL(c, chat(f_n)), |f_n - f_{n-1}| / |f_n|)
    every ``dtpl_every`` iterations (and the last) if dtpl_every > 0."""
    L = X.shape[0]
    P = X.shape[1]
    if rho is None:
        rho = np.asarray(X.sum(axis=1)).ravel()
    st = initial_state(spec.n_mat, P, L, spec.n_win, f0)
    hist: List[tuple] = []
    for it in range(n_iter):
        prev = st.f
        st = mocca_step(X, rho, st, c, spec, lam, precond, curvature)
        if dtpl_every and ((it + 1) % dtpl_every == 0 or it + 1 == n_iter):
            d = model.image_objective(X, st.f, c, spec)
            nf = np.linalg.norm(st.f)
            rel = np.linalg.norm(st.f - prev) / nf if nf > 0 else np.inf
            hist.append((it + 1, d, rel))
        if callback is not None:
            callback(it, st)
    return st, hist


def mocca_nested(X, c, spec, lam: float, n_outer: int, n_inner: int, precond: str = "block",
                 curvature: str = "clip", f0=None, rho=None, state: Optional[State] = None,
                 callback: Optional[Callable[[int, int, State], None]] = None):
    """MOCCA with nested loops (Sec. III names them as the remedy for the
    divergence a single inner iteration can show): ``n_outer`` expansion
    points, each the extrapolated iterate fbar at the start of its outer
    iteration, and ``n_inner`` CPPD steps on the fixed convex quadratic
    Q(K(f0) f) formed there (K, Sigma, T, r, D and u0 = K(f0) f0 all at f0).
    n_inner = 1 is ``mocca``.  Starts from ``state`` if given, else from f0
    (default 0) with y0 = 0; returns the final state.  callback(outer, inner,
    state) after every step."""
    L = X.shape[0]
    P = X.shape[1]
    if rho is None:
        rho = np.asarray(X.sum(axis=1)).ravel()
    st = state if state is not None else initial_state(spec.n_mat, P, L, spec.n_win, f0)
    for o in range(n_outer):
        expansion = st.fbar.copy()
        for j in range(n_inner):
            st = mocca_step(X, rho, st, c, spec, lam, precond, curvature, expansion=expansion)
            if callback is not None:
                callback(o, j, st)
    return st

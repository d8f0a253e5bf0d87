"""Counts model, data discrepancy and derivatives of Sec. II, FP64.

Arrays are ray-major: p [L, M] material line integrals (X f_m)_l, counts and
residuals [L, W].  The spectral tables come from ``synth.Spectral``:
mu [M, I], s [W, I] (rows sum to one, shared by all rays), n0 [W]; or from
``synth.RaySpectral`` with a response per ray, s [L, W, I] and n0 [L, W]
(the paper's per-detector-pixel spectra).

Pinned by: zero attenuation (window totals chat = N, A = B = s), the
monochromatic Beer-Lambert case, central finite differences of D_TPL for the
gradient and of the gradient for the Hessian, and the sign facts the paper
uses (C = A - B >= 0 elementwise).
"""
from __future__ import annotations

import numpy as np


# --- softexp (Sec. II): exp for arguments <= 0, its tangent line x + 1 above.
# softexp'' is taken from the x <= 0 branch at x = 0 (the paper's case split).

def softexp(x):
    x = np.asarray(x, dtype=np.float64)
    return np.where(x <= 0.0, np.exp(np.minimum(x, 0.0)), x + 1.0)


def softexp_d1(x):
    x = np.asarray(x, dtype=np.float64)
    return np.where(x <= 0.0, np.exp(np.minimum(x, 0.0)), 1.0)


def softexp_d2(x):
    x = np.asarray(x, dtype=np.float64)
    return np.where(x <= 0.0, np.exp(np.minimum(x, 0.0)), 0.0)


def energy_line_integrals(p, mu):
    """(Z f)_{l,i} = sum_{m,k} mu_{m,i} X_{l,k} f_{k,m} = sum_m mu_{m,i} p_{l,m}."""
    return np.asarray(p, dtype=np.float64) @ mu


def per_ray(spec) -> bool:
    return np.ndim(spec.s) == 3


def incident(spec):
    """N as [L or 1, W]."""
    n0 = np.asarray(spec.n0, dtype=np.float64)
    return n0 if n0.ndim == 2 else n0[None, :]


def window_sums(e, spec):
    """sum_i s_{w,i} e_{l,i} -> [L, W] (s shared or per ray)."""
    if per_ray(spec):
        return np.einsum("li,lwi->lw", e, spec.s)
    return e @ spec.s.T


def counts_model(p, spec):
    """chat_{w,l} of Eq. (finalModel): N_w sum_i s_{w,i} softexp(-(Zf)_{l,i})."""
    z = energy_line_integrals(p, spec.mu)
    return incident(spec) * window_sums(softexp(-z), spec)


def counts_model_standard(p, spec):
    """chat of Eq. (fullModel), plain exp (equal to Eq. finalModel when Zf >= 0)."""
    z = energy_line_integrals(p, spec.mu)
    return incident(spec) * window_sums(np.exp(-z), spec)


def dtpl_terms(c, chat):
    """Per-(l, w) terms of Eq. (DTPL): chat - c - c log(chat / c), with 0 log 0 = 0."""
    c = np.asarray(c, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        lg = np.where(c > 0.0, c * np.log(chat / np.where(c > 0.0, c, 1.0)), 0.0)
    return chat - c - lg


def dtpl(c, chat) -> float:
    return float(np.sum(dtpl_terms(c, chat)))


def residual(c, chat):
    """r_{w,l} = c_{w,l} - chat_{w,l}."""
    return np.asarray(c, dtype=np.float64) - chat


def matrices_AB(p, spec):
    """Per-ray blocks of A(f) and B(f) (Eq. aeq and the one after it).

    A and B are block-diagonal over rays (the identity I_{l,l'}); returns
    A[l, w, i] = s_{w,i} softexp'(-(Zf)_{l,i}) / sum_i' s_{w,i'} softexp(-(Zf)_{l,i'})
    and B with softexp'' in the numerator, plus g[l, w] (the denominator)."""
    z = energy_line_integrals(p, spec.mu)
    g = window_sums(softexp(-z), spec)                           # [L, W]
    S = spec.s if per_ray(spec) else spec.s[None, :, :]
    A = S * softexp_d1(-z)[:, None, :] / g[:, :, None]
    B = S * softexp_d2(-z)[:, None, :] / g[:, :, None]
    return A, B, g


def ray_jacobian_from_A(A, spec):
    """G_l = A_l mu^T in R^{W x M}: K(f)_{wl, mk} = G_l[w, m] X_{l,k} (K = A Z)."""
    return A @ spec.mu.T


def ray_jacobian(p, spec):
    A, _, _ = matrices_AB(p, spec)
    return ray_jacobian_from_A(A, spec)


def gradient_p(p, c, spec):
    """Per-ray gradient of L_TPL in p-space: (A mu^T)^T r  (the p_l part of
    Z^T A^T r; the image gradient is X^T of it)."""
    A, _, g = matrices_AB(p, spec)
    r = residual(c, incident(spec) * g)
    return np.einsum("lwi,mi,lw->lm", A, spec.mu, r)


def hessian_from_AB(A, B, g, c, spec):
    """Per-ray Hessian of L_TPL in p-space, the ray-l block of
    -Z^T diag(B^T r) Z + Z^T A^T diag(chat + r) A Z (Sec. II), as [L, M, M]."""
    chat = incident(spec) * g
    r = residual(c, chat)
    btr = np.einsum("lwi,lw->li", B, r)                          # (B^T r)_{l,i}
    term1 = -np.einsum("mi,li,ni->lmn", spec.mu, btr, spec.mu, optimize=True)
    am = A @ spec.mu.T                                           # (A Z) per ray, [L,W,M]
    term2 = np.einsum("lwm,lw,lwn->lmn", am, chat + r, am, optimize=True)
    return term1 + term2


def hessian_p(p, c, spec):
    A, B, g = matrices_AB(p, spec)
    return hessian_from_AB(A, B, g, c, spec)


def image_gradient(X, f, c, spec):
    """grad_f L_TPL = Z^T A^T r = X^T (G_l^T r_l), f as [M, n*n] -> [M, n*n]."""
    p = (X @ f.T)
    return (X.T @ gradient_p(p, c, spec)).T


def image_objective(X, f, c, spec) -> float:
    """L_TPL(f) = D_TPL(c, chat(f))."""
    return dtpl(c, counts_model(X @ f.T, spec))

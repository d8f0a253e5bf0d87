"""Step lengths of Sec. II: diagonal SPC (Pock-Chambolle) and the paper's
m-block-diagonal SPC, FP64.

Two routes compute the same numbers:

* ``*_dense``: the paper's formulas applied literally to an explicit K
  (rows (w, l), columns (m, k)); tiny problems only.
* ``*_factored``: K_{wl,mk} = G_l[w, m] X_{l,k} with X >= 0, so the sums over
  pixels collapse onto rho_l = (X 1)_l and the sums over rays become
  back-projections:  block  Sigma^-1_{wl} = lam rho_l |G_l[w,:]|,
  (T^-1)_k = (1/lam) sum_l X_{l,k} S_l with S_l = sum_w G_l[w]^T G_l[w] / |G_l[w]|;
  diagonal  Sigma^-1_{wl} = lam rho_l sum_m |G_l[w,m]|,
  T_{mk} = lam / sum_l X_{l,k} h_{l,m} with h_{l,m} = sum_w |G_l[w,m]|.

Pinned by: equality of the two routes on random tiny K (the factorisation is
exact), and positive semi-definiteness of M = [[T^-1, -K^T], [-K, Sigma^-1]],
the convergence condition the paper states for SPC CPPD.
"""
from __future__ import annotations

import numpy as np

# ------------------------------------------------------------------ dense K


def dense_K(G, X):
    """K[(w,l), (m,k)] = sum_{l',i} A_{wl,l'i} Z_{l'i,mk} = G_l[w,m] X_{l,k}.

    G: [L, W, M], X: dense [L, P].  Rows ordered w-major (w*L + l), columns
    m-major (m*P + k)."""
    L, W, M = G.shape
    P = X.shape[1]
    K = np.einsum("lwm,lk->wlmk", G, X)
    return K.reshape(W * L, M * P)


def diag_steps_dense(K, lam, n_mat):
    """Sigma_{wl} = (1/lam) / sum_{mk} |K|,  T_{mk} = lam / sum_{wl} |K|."""
    absK = np.abs(K)
    rs = absK.sum(axis=1)
    cs = absK.sum(axis=0)
    with np.errstate(divide="ignore"):
        sigma = np.where(rs > 0, (1.0 / lam) / rs, 0.0)
        tau = np.where(cs > 0, lam / cs, 0.0)
    return sigma, tau


def block_steps_dense(K, lam, n_mat):
    """(Sigma^-1)_{wl} = lam sum_k sqrt(sum_m K^2);
    (T^-1)_{k}[m,m'] = (1/lam) sum_{wl} K_{wl,mk} K_{wl,m'k} / sqrt(sum_m'' K^2_{wl,m''k})
    (0/0 taken as 0).  Returns Sigma^-1 [W*L] and T^-1 blocks [P, M, M]."""
    R = K.shape[0]
    P = K.shape[1] // n_mat
    Kr = K.reshape(R, n_mat, P)                       # [row, m, k]
    nrm = np.sqrt((Kr ** 2).sum(axis=1))              # [row, k]
    sigma_inv = lam * nrm.sum(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        wgt = np.where(nrm > 0, 1.0 / nrm, 0.0)
    tinv = np.einsum("rmk,rnk,rk->kmn", Kr, Kr, wgt) / lam
    return sigma_inv, tinv


def assemble_M(K, tinv_blocks=None, tau=None, sigma_inv=None, sigma=None):
    """Dense M = [[T^-1, -K^T], [-K, Sigma^-1]] (block or diagonal T)."""
    R, C = K.shape
    if tinv_blocks is not None:
        P, M, _ = tinv_blocks.shape
        Tinv = np.zeros((C, C))
        for k in range(P):
            idx = np.arange(M) * P + k
            Tinv[np.ix_(idx, idx)] = tinv_blocks[k]
    else:
        Tinv = np.diag(1.0 / tau)
    Sinv = np.diag(sigma_inv if sigma_inv is not None else 1.0 / sigma)
    return np.block([[Tinv, -K.T], [-K, Sinv]])


# ------------------------------------------------------------- factorised


def ray_block_terms(G):
    """|G_l[w,:]|_2 [L, W] and S_l = sum_w G_l[w]^T G_l[w] / |G_l[w]| [L, M, M]."""
    nrm = np.sqrt((G ** 2).sum(axis=2))
    with np.errstate(divide="ignore", invalid="ignore"):
        wgt = np.where(nrm > 0, 1.0 / nrm, 0.0)
    S = np.einsum("lwm,lwn,lw->lmn", G, G, wgt)
    return nrm, S


def block_steps_factored(G, X, rho, lam):
    """sigma [L, W] (0 where the ray misses the image) and T^-1 blocks [P, M, M]."""
    nrm, S = ray_block_terms(G)
    den = lam * rho[:, None] * nrm
    with np.errstate(divide="ignore"):
        sigma = np.where(den > 0, 1.0 / den, 0.0)
    M = G.shape[2]
    tinv = (X.T @ S.reshape(-1, M * M)).reshape(-1, M, M) / lam
    return sigma, tinv


def diag_steps_factored(G, X, rho, lam):
    """sigma [L, W] and tau [P, M] of diagonal SPC."""
    absG = np.abs(G)
    den = lam * rho[:, None] * absG.sum(axis=2)
    with np.errstate(divide="ignore"):
        sigma = np.where(den > 0, 1.0 / den, 0.0)
    h = absG.sum(axis=1)                              # [L, M]
    cs = X.T @ h                                      # [P, M]
    with np.errstate(divide="ignore"):
        tau = np.where(cs > 0, lam / cs, 0.0)
    return sigma, tau

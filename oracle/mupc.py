"""mu-preconditioning (mu-PC): MOCCA with diagonal SPC in a material basis
that is orthonormal in X-ray energy (Sec. I; Sec. II "Step lengths"), FP64.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and
bench.py's CPU baseline; never by the library or its binding.

The paper describes mu-PC as a change of material basis to attenuation
curves that are mutually orthogonal over energy, with diagonal SPC's step
lengths formed from K(f0) in the new basis, and leaves the transform itself
to its Ref. Barber2016b.  Reading taken here:

  * inner product over energy bins  <u, v> = sum_i w_i u_i v_i  with
    w_i = (1/W) sum_w s_{w,i}, the detected spectrum averaged over windows;
  * Gram-Schmidt of the attenuation rows mu_m(E_i) in material order gives
    mu~ = B mu with <mu~_j, mu~_k> = delta_jk, B lower triangular with a
    positive diagonal;
  * the attenuation map is unchanged: sum_m f_m mu_m = sum_j g_j mu~_j, i.e.
    f = B^T g; MOCCA with diagonal SPC runs on g with mu~ in place of mu and
    the maps are f = B^T g.

Pins (tests/test_oracle.py): orthonormality of mu~ under the weights; B
equals the inverse Cholesky factor of the weighted Gram matrix (the textbook
identity for Gram-Schmidt); the counts model is invariant under the change
of basis; the noiseless truth is a fixed point.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import mocca as _mocca


def energy_weights(spec) -> np.ndarray:
    """w_i = (1/W) sum_w s_{w,i} (sums to 1 when every row of s does)."""
    return np.asarray(spec.s, dtype=np.float64).mean(axis=0)


def mu_pc_basis(spec):
    """Gram-Schmidt of the rows of mu under <u, v>_w.  Returns (B, mu~) with
    mu~ = B mu orthonormal."""
    w = energy_weights(spec)
    mu = np.asarray(spec.mu, dtype=np.float64)
    M = mu.shape[0]
    B = np.zeros((M, M))
    Q = np.zeros_like(mu)
    for j in range(M):
        v = mu[j].copy()
        b = np.zeros(M)
        b[j] = 1.0
        for k in range(j):
            proj = float(np.sum(w * mu[j] * Q[k]))   # <mu_j, q_k>
            v = v - proj * Q[k]
            b = b - proj * B[k]
        nrm = float(np.sqrt(np.sum(w * v * v)))
        Q[j] = v / nrm
        B[j] = b / nrm
    return B, Q


def transformed_spectral(spec):
    """The spectral description with mu~ in place of mu, and B."""
    B, Q = mu_pc_basis(spec)
    return dataclasses.replace(spec, mu=Q), B


def maps_from_basis(g, B):
    """f = B^T g for maps g [M][P]."""
    return B.T @ np.asarray(g, dtype=np.float64)


def basis_from_maps(f, B):
    """g = B^-T f."""
    return np.linalg.solve(B.T, np.asarray(f, dtype=np.float64))


def mocca_mu_pc(X, c, spec, lam: float, n_iter: int, curvature: str = "clip", f0=None, dtpl_every: int = 0):
    """n_iter MOCCA iterations with diagonal SPC in the mu-PC basis from f0
    (default 0).  Returns (f [M][P], state in the g basis, history, B)."""
    spec_t, B = transformed_spectral(spec)
    g0 = None if f0 is None else basis_from_maps(f0, B)
    st, hist = _mocca.mocca(X, c, spec_t, lam, n_iter, "diag", curvature, f0=g0, dtpl_every=dtpl_every)
    return maps_from_basis(st.f, B), st, hist, B

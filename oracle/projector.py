"""Discrete X-ray projection X_{l,k} of Eq. (fullModel), FP64.

X_{l,k} is the length of ray l inside pixel k (the line-intersection model:
the paper only calls X "X-ray projection along ray l"; the exact chord length
is the reading taken here).  The matrix is built with Siddon's method: the
parametric positions where the ray crosses the grid lines are merged and
sorted, and every segment between consecutive crossings belongs to the pixel
containing its midpoint.  Rows are rays l = v*n_bins + d, columns are pixels
k = iy*n + ix.

Pinned by: a brute-force Liang-Barsky clip of every (ray, pixel) pair on tiny
grids, the closed-form chord of the whole image square (row sums), analytic
chords through disks, and the 90-degree rotation symmetry of the scan.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np
import scipy.sparse as sp


def view_cos_sin(beta):
    """cos and sin of the view angles, taken exactly (0 and +-1) where the
    angle is a multiple of pi/2: the rays of such a view through the
    detector centre are exactly parallel to an image axis, which FP64's
    cos(pi/2) ~ 6e-17 would turn by rounding alone."""
    cb, sb = np.cos(beta), np.sin(beta)
    zc, zs = np.abs(cb) < 1e-12, np.abs(sb) < 1e-12
    return np.where(zc, 0.0, np.where(zs, np.sign(cb), cb)), np.where(zs, 0.0, np.where(zc, np.sign(sb), sb))


def ray_endpoints(geom, views: Optional[Sequence[int]] = None):
    """Source S and detector-bin centre P of every ray, shape [n_rays, 2] each.

    Rays are ordered view-major, bin-minor, over ``views`` (default: all)."""
    v = np.arange(geom.n_views) if views is None else np.asarray(views, dtype=np.int64)
    beta = geom.view0_rad + geom.arc_rad * v / geom.n_views
    cb, sb = view_cos_sin(beta)
    u = (np.arange(geom.n_bins) - (geom.n_bins - 1) / 2.0) * geom.bin_cm
    s = np.stack([geom.sid_cm * cb, geom.sid_cm * sb], axis=1)                      # [V,2]
    dc = np.stack([-(geom.sdd_cm - geom.sid_cm) * cb, -(geom.sdd_cm - geom.sid_cm) * sb], axis=1)
    eu = np.stack([-sb, cb], axis=1)
    p = dc[:, None, :] + u[None, :, None] * eu[:, None, :]                        # [V,D,2]
    s_all = np.broadcast_to(s[:, None, :], p.shape)
    return s_all.reshape(-1, 2).copy(), p.reshape(-1, 2).copy()


def _siddon_chunk(S, P, n, pix):
    """Siddon segments of a chunk of rays: (ray_in_chunk, pixel, length)."""
    half = n * pix / 2.0
    planes = (np.arange(n + 1) - n / 2.0) * pix
    d = P - S
    length = np.hypot(d[:, 0], d[:, 1])
    with np.errstate(divide="ignore", invalid="ignore"):
        ax = (planes[None, :] - S[:, :1]) / d[:, :1]
        ay = (planes[None, :] - S[:, 1:]) / d[:, 1:]
        ax_lo = np.minimum(ax[:, 0], ax[:, -1]); ax_hi = np.maximum(ax[:, 0], ax[:, -1])
        ay_lo = np.minimum(ay[:, 0], ay[:, -1]); ay_hi = np.maximum(ay[:, 0], ay[:, -1])
    # a ray parallel to an axis sees the whole (or none) of that axis' slab
    inx = (S[:, 0] > -half) & (S[:, 0] < half)
    iny = (S[:, 1] > -half) & (S[:, 1] < half)
    par_x = d[:, 0] == 0.0
    par_y = d[:, 1] == 0.0
    ax_lo = np.where(par_x, np.where(inx, -np.inf, np.inf), ax_lo)
    ax_hi = np.where(par_x, np.where(inx, np.inf, -np.inf), ax_hi)
    ay_lo = np.where(par_y, np.where(iny, -np.inf, np.inf), ay_lo)
    ay_hi = np.where(par_y, np.where(iny, np.inf, -np.inf), ay_hi)
    a_min = np.maximum(np.maximum(ax_lo, ay_lo), 0.0)
    a_max = np.minimum(np.minimum(ax_hi, ay_hi), 1.0)
    hit = a_max > a_min
    allv = np.concatenate([ax, ay, a_min[:, None], a_max[:, None]], axis=1)
    allv = np.where(np.isfinite(allv), allv, a_max[:, None])
    allv = np.clip(allv, a_min[:, None], a_max[:, None])
    allv.sort(axis=1)
    seg = np.diff(allv, axis=1)                                    # [R, 2n+3]
    mid = 0.5 * (allv[:, 1:] + allv[:, :-1])
    xm = S[:, :1] + mid * d[:, :1]
    ym = S[:, 1:] + mid * d[:, 1:]
    # pixels are half-open, [edge_i, edge_i+1): a segment lying on a shared
    # grid line (a ray exactly on an edge) belongs to the pixel on its + side
    ix = np.floor(xm / pix + 0.5 * n).astype(np.int64)
    iy = np.floor(ym / pix + 0.5 * n).astype(np.int64)
    keep = (seg > 0.0) & hit[:, None]
    r_idx = np.broadcast_to(np.arange(S.shape[0])[:, None], seg.shape)[keep]
    ix, iy = ix[keep], iy[keep]
    assert ix.size == 0 or (ix.min() >= 0 and ix.max() < n and iy.min() >= 0 and iy.max() < n)
    lens = (seg * length[:, None])[keep]
    return r_idx, iy * n + ix, lens


def system_matrix(geom, views: Optional[Sequence[int]] = None, chunk: int = 2048) -> sp.csr_matrix:
    """X as a CSR matrix [n_rays(views), n*n] of chord lengths in cm."""
    S, P = ray_endpoints(geom, views)
    n = geom.n
    rows, cols, vals = [], [], []
    for c0 in range(0, S.shape[0], chunk):
        r, k, l = _siddon_chunk(S[c0:c0 + chunk], P[c0:c0 + chunk], n, geom.pixel_cm)
        rows.append(r + c0); cols.append(k); vals.append(l)
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    vals = np.concatenate(vals) if vals else np.zeros(0)
    return sp.csr_matrix((vals, (rows, cols)), shape=(S.shape[0], n * n))


def clip_chord(S, P, x_lo, x_hi, y_lo, y_hi):
    """Length of segment S->P inside the box [x_lo,x_hi] x [y_lo,y_hi]
    (Liang-Barsky clipping), vectorised over broadcastable arguments."""
    S = np.asarray(S, dtype=np.float64); P = np.asarray(P, dtype=np.float64)
    dx, dy = P[..., 0] - S[..., 0], P[..., 1] - S[..., 1]
    t0 = np.zeros(np.broadcast(dx, x_lo, y_lo).shape)
    t1 = np.ones_like(t0)
    for pk, qk in ((-dx, S[..., 0] - x_lo), (dx, x_hi - S[..., 0]),
                   (-dy, S[..., 1] - y_lo), (dy, y_hi - S[..., 1])):
        pk = np.broadcast_to(pk, t0.shape); qk = np.broadcast_to(qk, t0.shape)
        with np.errstate(divide="ignore", invalid="ignore"):
            r = qk / pk
        neg, pos, par = pk < 0, pk > 0, pk == 0
        t0 = np.where(neg, np.maximum(t0, r), t0)
        t1 = np.where(pos, np.minimum(t1, r), t1)
        t1 = np.where(par & (qk < 0), -1.0, t1)   # parallel and outside
    return np.maximum(t1 - t0, 0.0) * np.hypot(dx, dy)


def dense_matrix_bruteforce(geom) -> np.ndarray:
    """X by clipping every ray against every pixel square (tiny grids only)."""
    S, P = ray_endpoints(geom)
    n, pix = geom.n, geom.pixel_cm
    edges = (np.arange(n + 1) - n / 2.0) * pix
    xl = np.tile(edges[:-1], n); xh = np.tile(edges[1:], n)
    yl = np.repeat(edges[:-1], n); yh = np.repeat(edges[1:], n)
    return clip_chord(S[:, None, :], P[:, None, :], xl[None], xh[None], yl[None], yh[None])


def pixel_column(geom, ix: int, iy: int, views: Optional[Sequence[int]] = None) -> np.ndarray:
    """Column k = (ix, iy) of X over all rays, by direct clipping."""
    S, P = ray_endpoints(geom, views)
    pix = geom.pixel_cm
    x0 = (ix - geom.n / 2.0) * pix
    y0 = (iy - geom.n / 2.0) * pix
    return clip_chord(S, P, x0, x0 + pix, y0, y0 + pix)


def square_chord(geom, views: Optional[Sequence[int]] = None) -> np.ndarray:
    """Closed form of X.1: chord of every ray through the whole image square."""
    S, P = ray_endpoints(geom, views)
    h = geom.n * geom.pixel_cm / 2.0
    return clip_chord(S, P, -h, h, -h, h)


def disk_chord(geom, cx: float, cy: float, radius: float, views=None) -> np.ndarray:
    """Analytic chord 2*sqrt(r^2 - d^2) of every ray through a disk (d = distance
    from the disk centre to the ray's line)."""
    S, P = ray_endpoints(geom, views)
    d = P - S
    nrm = np.hypot(d[:, 0], d[:, 1])
    dist = np.abs((cx - S[:, 0]) * d[:, 1] - (cy - S[:, 1]) * d[:, 0]) / nrm
    return 2.0 * np.sqrt(np.maximum(radius ** 2 - dist ** 2, 0.0)), dist

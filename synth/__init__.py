"""Seeded synthetic inputs for one-step three-material spectral CT.

This module produces the *inputs* of the reconstruction problem stated in
Sec. II (Methods) of Sidky, Barber, Gilat-Schmidt and Pan, "Three material
decomposition for spectral computed tomography enabled by block-diagonal
step-preconditioning" (arXiv 1801.06263): the fan-beam scan geometry, the
material attenuation table mu_{m,i} of the material expansion (Eq. matdecomp),
the normalised window responses s_{w,i} and incident counts N_w of the
discrete counts model (Eq. fullModel), a disk phantom f and the Poisson draw
of measured counts c.

It holds none of the method's arithmetic: no projector, no counts model, no
derivative and no step length.  Both the FP64 oracle and the GPU library read
what it produces; measured counts need a mean (the counts model evaluated at
the phantom), which the caller computes with its own side and passes to
``poisson_counts``.

The paper's own bench-top spectra, rods phantom and detector geometry are not
published, so these synthetic stand-ins take their place (four overlapping
windows, three materials PMMA / Al / Gd, a PMMA cylinder with Al and Gd
inserts, Sec. III).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np
from scipy.special import erf

MATERIALS = ("PMMA", "Al", "Gd")

# photo-electric / Compton coefficients (cm^-1 at 30 keV) of the three
# synthetic materials; the Gd photo-electric term jumps x5 at its K edge.
_ATTEN_AB = ((0.02, 0.20), (0.35, 0.38), (30.0, 0.9))
GD_K_EDGE_KEV = 50.2
GD_K_JUMP = 5.0


@dataclasses.dataclass(frozen=True)
class Geometry:
    """2-D fan beam with a flat detector, image centred on the isocentre.

    Image: ``n`` x ``n`` square pixels of side ``pixel_cm``; array layout
    ``[ny][nx]`` (x fastest), pixel (ix, iy) centred at
    ((ix-(n-1)/2) * pixel_cm, (iy-(n-1)/2) * pixel_cm).
    View v: source angle beta_v = view0_rad + arc_rad * v / n_views, source at
    sid_cm * (cos beta, sin beta), detector centre at
    -(sdd_cm - sid_cm) * (cos beta, sin beta), detector axis (-sin beta, cos beta),
    bin d centred at u_d = (d - (n_bins-1)/2) * bin_cm.
    Sinogram layout ``[n_views][n_bins]`` (bin fastest); ray l = v*n_bins + d.
    """

    n: int
    pixel_cm: float
    n_views: int
    n_bins: int
    sid_cm: float
    sdd_cm: float
    bin_cm: float
    view0_rad: float = 0.0
    arc_rad: float = 2.0 * math.pi

    @property
    def fov_cm(self) -> float:
        return self.n * self.pixel_cm

    @property
    def n_rays(self) -> int:
        return self.n_views * self.n_bins


def covering_bin_pitch(fov_cm: float, sid_cm: float, sdd_cm: float, n_bins: int) -> float:
    """Flat-detector pitch whose fan just covers the image square's circumcircle."""
    rc = fov_cm / math.sqrt(2.0)
    return 2.0 * sdd_cm * math.tan(math.asin(rc / sid_cm)) / n_bins


def make_geometry(n: int, fov_cm: float, n_views: int, n_bins: int,
                  sid_cm: float = 50.0, sdd_cm: float = 100.0,
                  bin_cm: Optional[float] = None) -> Geometry:
    if bin_cm is None:
        bin_cm = covering_bin_pitch(fov_cm, sid_cm, sdd_cm, n_bins)
    return Geometry(n=n, pixel_cm=fov_cm / n, n_views=n_views, n_bins=n_bins,
                    sid_cm=sid_cm, sdd_cm=sdd_cm, bin_cm=bin_cm)


# ----------------------------------------------------------------- physics

def klein_nishina(e_kev):
    """Total Klein-Nishina cross-section per electron (units of 2*pi*r_e^2)."""
    eps = np.asarray(e_kev, dtype=np.float64) / 511.0
    l2 = np.log1p(2.0 * eps)
    return ((1.0 + eps) / eps ** 2 * (2.0 * (1.0 + eps) / (1.0 + 2.0 * eps) - l2 / eps)
            + l2 / (2.0 * eps) - (1.0 + 3.0 * eps) / (1.0 + 2.0 * eps) ** 2)


def attenuation_table(energies_kev) -> np.ndarray:
    """mu[m, i] in cm^-1 per unit material fraction, materials PMMA, Al, Gd."""
    e = np.asarray(energies_kev, dtype=np.float64)
    kn = klein_nishina(e) / klein_nishina(30.0)
    mu = np.empty((3, e.size))
    for m, (a, b) in enumerate(_ATTEN_AB):
        photo = a * (e / 30.0) ** -3
        if MATERIALS[m] == "Gd":
            photo = photo * np.where(e > GD_K_EDGE_KEV, GD_K_JUMP, 1.0)
        mu[m] = photo + b * kn
    return mu


def kramers_photons(energies_kev, kvp: float) -> np.ndarray:
    """Kramers bremsstrahlung photon-number spectrum, (kVp - E)/E, zero above kVp."""
    e = np.asarray(energies_kev, dtype=np.float64)
    return np.where(e < kvp, (kvp - e) / e, 0.0)


def window_responses(energies_kev, edges_kev, blur_kev: float) -> np.ndarray:
    """Box windows [lo, hi] blurred by a Gaussian of std ``blur_kev``: R[w, i]."""
    e = np.asarray(energies_kev, dtype=np.float64)
    r = np.empty((len(edges_kev), e.size))
    k = math.sqrt(2.0) * blur_kev
    for w, (lo, hi) in enumerate(edges_kev):
        r[w] = 0.5 * (erf((e - lo) / k) - erf((e - hi) / k))
    return r


def spectral_response(energies_kev, kvp: float, edges_kev, blur_kev: float) -> np.ndarray:
    """Normalised window responses s[w, i] >= 0 with sum_i s[w, i] = 1."""
    s = kramers_photons(energies_kev, kvp)[None, :] * window_responses(energies_kev, edges_kev, blur_kev)
    return s / s.sum(axis=1, keepdims=True)


@dataclasses.dataclass(frozen=True)
class Spectral:
    mu: np.ndarray   # [M][I]
    s: np.ndarray    # [W][I], rows sum to one
    n0: np.ndarray   # [W] incident photons per ray per window

    @property
    def n_mat(self) -> int:
        return self.mu.shape[0]

    @property
    def n_win(self) -> int:
        return self.s.shape[0]

    @property
    def n_energy(self) -> int:
        return self.s.shape[1]


def make_spectral(e_lo: int, e_hi: int, kvp: float, i0: float,
                  edges=None, blur_kev: float = 5.0, e_step: int = 1) -> Spectral:
    """Tables on energies e_lo, e_lo + e_step, ..., <= e_hi (keV, bin centres)."""
    energies = np.arange(e_lo, e_hi + 1, e_step, dtype=np.float64)
    if edges is None:
        edges = ((20.0, 35.0), (35.0, 50.0), (50.0, 65.0), (65.0, float(kvp)))
    s = spectral_response(energies, kvp, edges, blur_kev)
    return Spectral(mu=attenuation_table(energies), s=s, n0=np.full(len(edges), float(i0)))


@dataclasses.dataclass(frozen=True)
class DetectorSpectral:
    """Per-detector-bin window responses and incident counts (a calibrated
    photon-counting detector): the same bin has the same response in every
    view."""
    mu: np.ndarray   # [M][I]
    s: np.ndarray    # [D][W][I], each (d, w) row sums to one
    n0: np.ndarray   # [D][W] incident photons per ray per window

    @property
    def n_mat(self) -> int:
        return self.mu.shape[0]

    @property
    def n_bins(self) -> int:
        return self.s.shape[0]

    @property
    def n_win(self) -> int:
        return self.s.shape[1]

    @property
    def n_energy(self) -> int:
        return self.s.shape[2]

    def for_rays(self, n_views: int) -> "RaySpectral":
        """The same tables per ray l = v * n_bins + d."""
        return RaySpectral(mu=self.mu, s=np.tile(self.s, (n_views, 1, 1)), n0=np.tile(self.n0, (n_views, 1)))


@dataclasses.dataclass(frozen=True)
class RaySpectral:
    """Per-ray window responses s [L][W][I] and incident counts n0 [L][W]."""
    mu: np.ndarray
    s: np.ndarray
    n0: np.ndarray

    @property
    def n_mat(self) -> int:
        return self.mu.shape[0]

    @property
    def n_win(self) -> int:
        return self.s.shape[1]

    @property
    def n_energy(self) -> int:
        return self.s.shape[2]


def make_detector_spectral(n_bins: int, e_lo: int, e_hi: int, kvp: float, i0: float, seed: int,
                           edge_jitter_kev: float = 1.5, blur_kev=(4.0, 6.0), gain_jitter: float = 0.1,
                           edges=None, e_step: int = 1) -> DetectorSpectral:
    """Bin-to-bin variation of a photon-counting detector: every bin's window
    thresholds shifted by N(0, edge_jitter_kev) (kept increasing), its energy
    blur drawn uniformly from blur_kev, and its incident counts per window
    scaled by 1 + gain_jitter N(0, 1) (clipped to [0.5, 1.5])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    energies = np.arange(e_lo, e_hi + 1, e_step, dtype=np.float64)
    if edges is None:
        edges = ((20.0, 35.0), (35.0, 50.0), (50.0, 65.0), (65.0, float(kvp)))
    thr = np.array([lo for lo, _ in edges] + [edges[-1][1]], dtype=np.float64)
    W = len(edges)
    s = np.empty((n_bins, W, energies.size))
    n0 = np.empty((n_bins, W))
    for d in range(n_bins):
        t = thr.copy()
        t[:-1] += rng.normal(0.0, edge_jitter_kev, W)   # the top of the last window stays at kVp
        t = np.maximum.accumulate(t + np.arange(W + 1) * 1e-6)
        blur = rng.uniform(blur_kev[0], blur_kev[1])
        s[d] = spectral_response(energies, kvp, list(zip(t[:-1], t[1:])), blur)
        n0[d] = i0 * np.clip(1.0 + gain_jitter * rng.standard_normal(W), 0.5, 1.5)
    return DetectorSpectral(mu=attenuation_table(energies), s=s, n0=n0)


@dataclasses.dataclass(frozen=True)
class ModulatedSpectral:
    """Window responses (shared [W][I] or per detector bin [D][W][I]) with
    incident counts that vary from ray to ray: n0 [L][W] (the N_{w,l} of
    Eq. fullModel in full), n0_nominal the counts without modulation ([W] or
    [D][W])."""
    mu: np.ndarray
    s: np.ndarray
    n0: np.ndarray
    n0_nominal: np.ndarray

    @property
    def n0_ray(self) -> np.ndarray:
        return self.n0

    @property
    def n_mat(self) -> int:
        return self.mu.shape[0]

    @property
    def n_win(self) -> int:
        return self.s.shape[-2]

    @property
    def n_energy(self) -> int:
        return self.s.shape[-1]


def tube_modulation(geom: Geometry, depth: float = 0.3, bowtie: float = 0.25, seed: int = 0) -> np.ndarray:
    """Relative incident intensity of every ray, [L] (view-major): a tube
    current modulated with the view angle, 1 + depth cos(2 beta + phase) (as
    for an elliptical patient), times a bowtie filter that attenuates the fan
    towards its edges, 1 - bowtie (u / u_max)^2, times 1% ray-to-ray jitter
    from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    beta = geom.view0_rad + geom.arc_rad * np.arange(geom.n_views) / geom.n_views
    phase = rng.uniform(0.0, 2.0 * math.pi)
    tube = 1.0 + depth * np.cos(2.0 * beta + phase)
    u = (np.arange(geom.n_bins) - 0.5 * (geom.n_bins - 1)) / (0.5 * max(geom.n_bins - 1, 1))
    bow = 1.0 - bowtie * u ** 2
    jitter = 1.0 + 0.01 * rng.standard_normal((geom.n_views, geom.n_bins))
    return (tube[:, None] * bow[None, :] * jitter).reshape(-1)


def modulated_spectral(spec, geom: Geometry, seed: int = 0, **kw) -> ModulatedSpectral:
    """spec (Spectral or DetectorSpectral) with its incident counts scaled
    per ray by tube_modulation (the same factor in every window)."""
    rel = tube_modulation(geom, seed=seed, **kw)
    n0 = np.asarray(spec.n0, dtype=np.float64)
    base = np.tile(n0, (geom.n_views, 1)) if n0.ndim == 2 else np.broadcast_to(n0, (rel.size, n0.size))
    return ModulatedSpectral(mu=spec.mu, s=spec.s, n0=base * rel[:, None], n0_nominal=n0)


# ----------------------------------------------------------------- phantom

def disk_phantom(n: int, fov_cm: float, disks: List[Tuple[float, float, float, Tuple[float, float, float]]],
                 background: Tuple[float, float, Tuple[float, float, float]], supersample: int = 8) -> np.ndarray:
    """Material maps f[m, iy, ix] as area fractions by supersample^2 sampling.

    ``background`` = (radius, 0, values) of a centred disk; each disk in ``disks``
    = (x, y, radius, values) overrides the background where it lies.
    """
    pix = fov_cm / n
    sub = (np.arange(n * supersample) + 0.5) / supersample * pix - fov_cm / 2.0
    xx, yy = np.meshgrid(sub, sub)  # [y][x]
    f = np.zeros((3, n * supersample, n * supersample))
    br, _, bval = background
    inside = xx ** 2 + yy ** 2 < br ** 2
    for m in range(3):
        f[m][inside] = bval[m]
    for (cx, cy, r, val) in disks:
        inside = (xx - cx) ** 2 + (yy - cy) ** 2 < r ** 2
        for m in range(3):
            f[m][inside] = val[m]
    return f.reshape(3, n, supersample, n, supersample).mean(axis=(2, 4))


def inserts_phantom(n: int, fov_cm: float, gd_fractions=(0.002, 0.005, 0.010), scale: float = 1.0) -> np.ndarray:
    """PMMA disk (r = 9 cm * scale) with 4 Al and 3 Gd-in-PMMA inserts (r = 1 cm * scale)."""
    disks = []
    for j in range(7):
        ang = 2.0 * math.pi * j / 7.0
        cx, cy = 5.0 * scale * math.cos(ang), 5.0 * scale * math.sin(ang)
        val = (0.0, 1.0, 0.0) if j < 4 else (1.0, 0.0, gd_fractions[j - 4])
        disks.append((cx, cy, 1.0 * scale, val))
    return disk_phantom(n, fov_cm, disks, (9.0 * scale, 0.0, (1.0, 0.0, 0.0)))


def random_phantom(n: int, fov_cm: float, seed: int) -> np.ndarray:
    """Slice of the batched mix: PMMA disk r = 0.45 FOV with 4 Al and 3 Gd inserts
    (r = 0.05 FOV) at random non-overlapping positions within 0.35 FOV, Gd
    fractions uniform in [0.001, 0.02]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r_ins = 0.05 * fov_cm
    centres: List[Tuple[float, float]] = []
    while len(centres) < 7:
        rad = 0.35 * fov_cm * math.sqrt(rng.uniform())
        ang = rng.uniform(0.0, 2.0 * math.pi)
        c = (rad * math.cos(ang), rad * math.sin(ang))
        if all((c[0] - o[0]) ** 2 + (c[1] - o[1]) ** 2 > (2.2 * r_ins) ** 2 for o in centres):
            centres.append(c)
    gd = rng.uniform(0.001, 0.02, size=3)
    disks = []
    for j, (cx, cy) in enumerate(centres):
        val = (0.0, 1.0, 0.0) if j < 4 else (1.0, 0.0, float(gd[j - 4]))
        disks.append((cx, cy, r_ins, val))
    return disk_phantom(n, fov_cm, disks, (0.45 * fov_cm, 0.0, (1.0, 0.0, 0.0)))


def poisson_counts(mean: np.ndarray, seed: int) -> np.ndarray:
    """Measured counts c ~ Poisson(mean), PCG64(seed), returned as float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.poisson(np.asarray(mean, dtype=np.float64)).astype(np.float64)


# ----------------------------------------------------------------- configs

@dataclasses.dataclass(frozen=True)
class Problem:
    name: str
    geom: Geometry
    spec: Spectral
    f_true: np.ndarray   # [3][n][n]
    seed: int


def _problem(name: str, n: int, fov: float, views: int, bins: int, e_hi: int, kvp: float,
             i0: float, scale: float, seed: int) -> Problem:
    geom = make_geometry(n, fov, views, bins)
    spec = make_spectral(20, e_hi, kvp, i0)
    return Problem(name, geom, spec, inserts_phantom(n, fov, scale=scale), seed)


def problem(name: str) -> Problem:
    """The named workloads.

    tiny   : 64^2 over 20 cm, 64 views x 128 bins, 100 energies 20..119 keV, 120 kVp, I0 1e5
    medium : 256^2 over 20 cm, 256 views x 512 bins, same physics
    large  : 512^2 over 40 cm, 720 views x 1024 bins, 120 energies 20..139 keV, 140 kVp, I0 1e6
    """
    if name == "tiny":
        return _problem(name, 64, 20.0, 64, 128, 119, 120.0, 1e5, 1.0, 1801)
    if name == "medium":
        return _problem(name, 256, 20.0, 256, 512, 119, 120.0, 1e5, 1.0, 1802)
    if name == "large":
        return _problem(name, 512, 40.0, 720, 1024, 139, 140.0, 1e6, 2.0, 1803)
    raise KeyError(name)


BATCH_PIXEL_CM = 0.078125
BATCH_SIZES = (128, 256, 384, 512)


def batch_slice(size: int, slice_id: int) -> Problem:
    """One slice of the mixed-size batch: size^2 pixels of 0.078125 cm,
    round(1.4 size) views x 2 size bins, 140 kVp / 120 energies / I0 1e6."""
    fov = size * BATCH_PIXEL_CM
    geom = make_geometry(size, fov, int(round(1.4 * size)), 2 * size)
    spec = make_spectral(20, 139, 140.0, 1e6)
    return Problem(f"slice{slice_id}_{size}", geom, spec, random_phantom(size, fov, 3000 + slice_id), 3000 + slice_id)


def batch_mix(n_per_size: int = 6) -> List[Problem]:
    out = []
    sid = 0
    for size in BATCH_SIZES:
        for _ in range(n_per_size):
            out.append(batch_slice(size, sid))
            sid += 1
    return out

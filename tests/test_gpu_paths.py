"""Kernel paths the standard workloads do not reach, held to the same bars as
test_gpu_parity.py:

- the back-projector's wide path: a 16 x 16 tile whose detector shadow spans
  more bins than a staging slot of the grouped path (62) is staged one view
  at a time, in chunks of 128 bins when the shadow is wider still.  A 32^2
  image over 20 cm seen by 400 bins puts up to ~230 bins under one tile;
- the spectral dual step's vector energy sums: the matrix-core sums stage the
  energy table (padded to a multiple of 8 energies) in 64 KiB of LDS, so up to
  336 energies; 337 and more take the vector path.  33 energies leave 7 zero
  rows in the padded table, 336 fill it exactly;
- a batch holding a wide-shadow scan and a 337-energy scan beside the tiny
  scan: every slot bit-identical to its scan run alone.

Bars: sinograms and back-projections as in test_gpu_parity.py (1e-5 of the
sum of |terms|); maps and duals after the stated iterations within 1e-3
relative L2 of the FP64 oracle; batched slots bit-exact.
"""
import math
import warnings

import numpy as np
import pytest

import synth
from helpers import dev, host, normwise, sino
from oracle import model, mocca as omocca, projector as pj

warnings.filterwarnings("ignore", category=RuntimeWarning)
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

WIDE = synth.make_geometry(32, 20.0, 16, 400)
WIDE_OFFSET = synth.Geometry(n=30, pixel_cm=0.6, n_views=13, n_bins=333, sid_cm=45.0, sdd_cm=95.0, bin_cm=0.09,
                             view0_rad=0.41, arc_rad=math.pi)
SPEC = synth.make_spectral(20, 119, 120.0, 1e5, e_step=5)


def max_tile_shadow_bins(geom, tile=16):
    """Largest detector shadow (bins, plus a 3-bin margin) of a 16 x 16 pixel
    tile over all views: the quantity that sends a scan down the wide path
    when it exceeds 62."""
    h = geom.pixel_cm
    c0 = 0.5 * (geom.n - 1)
    sid = geom.sid_cm / h
    scale = geom.sdd_cm / geom.bin_cm
    nt = (geom.n + tile - 1) // tile
    out = 0.0
    for v in range(geom.n_views):
        beta = geom.view0_rad + geom.arc_rad * v / geom.n_views
        cb, sb = math.cos(beta), math.sin(beta)
        for ty in range(nt):
            for tx in range(nt):
                ts = []
                for k in range(4):
                    X = tx * tile - c0 - 0.5 + (tile if k & 1 else 0)
                    Y = ty * tile - c0 - 0.5 + (tile if k & 2 else 0)
                    ts.append((-sb * X + cb * Y) / (sid - cb * X - sb * Y))
                out = max(out, (max(ts) - min(ts)) * scale + 3.0)
    return out


def spectral_with(n_energy):
    """120 kVp spectrum and PMMA/Al/Gd table on n_energy bins spread evenly
    over 20..119 keV (the tiny workload's physics at another resolution)."""
    e = np.linspace(20.0, 119.0, n_energy)
    edges = ((20.0, 35.0), (35.0, 50.0), (50.0, 65.0), (65.0, 120.0))
    return synth.Spectral(mu=synth.attenuation_table(e), s=synth.spectral_response(e, 120.0, edges, 5.0),
                          n0=np.full(4, 1e5))


def plan_for(geom, spec):
    from paper_1801_06263_amd import Plan
    return Plan(geom, spec)


def oracle_counts(geom, spec, f_true, seed):
    X = pj.system_matrix(geom)
    return X, synth.poisson_counts(model.counts_model(X @ f_true.reshape(3, -1).T, spec), seed)


def assert_trajectory(plan, geom, X, c, spec, lam, n_it, tag):
    from paper_1801_06263_amd import Params
    ref, _ = omocca.mocca(X, c, spec, lam, n_it, "block", "clip")
    st = plan.new_state(dev(sino(c, geom.n_views, geom.n_bins)))
    plan.mocca_iterate(st, Params(lam, "block", "clip", True), n_it)
    f = host(st.f).reshape(3, -1)
    for m in range(3):
        rel = np.linalg.norm(f[m] - ref.f[m]) / np.linalg.norm(ref.f[m])
        print(f"{tag} material {m}: rel L2 {rel:.2e}")
        assert rel <= 1e-3, (tag, m, rel)
    y = host(st.y).reshape(4, -1).T
    rel_y = np.linalg.norm(y - ref.y) / np.linalg.norm(ref.y)
    print(f"{tag} dual rel L2 {rel_y:.2e}")
    assert rel_y <= 1e-3, (tag, rel_y)


# ---------------------------------------------------------------- wide shadows

@pytest.mark.parametrize("geom", [WIDE, WIDE_OFFSET], ids=["wide", "wide_offset"])
def test_wide_geometries_take_the_chunked_path(geom):
    assert max_tile_shadow_bins(geom) > 128 + 3


@pytest.mark.parametrize("geom", [WIDE, WIDE_OFFSET], ids=["wide", "wide_offset"])
def test_wide_back_projection_parity(geom):
    plan = plan_for(geom, SPEC)
    X = pj.system_matrix(geom)
    rng = np.random.default_rng(geom.n_bins)
    for nch in (9, 3, 1):
        q = rng.standard_normal((nch, geom.n_views, geom.n_bins)).astype(np.float32)
        b = host(plan.back_project(dev(q))).reshape(nch, -1)
        ref = (X.T @ q.reshape(nch, -1).astype(np.float64).T).T
        mag = (abs(X).T @ np.abs(q.reshape(nch, -1)).astype(np.float64).T).T
        assert np.abs(b - ref).max() <= 1e-5 * mag.max(), nch
    f = np.abs(rng.standard_normal((3, geom.n, geom.n))).astype(np.float32)
    p = host(plan.forward_project(dev(f))).reshape(3, -1)
    assert normwise(p, (X @ f.reshape(3, -1).astype(np.float64).T).T) <= 1e-5


def test_wide_mocca_trajectory_parity():
    geom = WIDE
    X, c = oracle_counts(geom, SPEC, synth.inserts_phantom(geom.n, 20.0), 21)
    assert_trajectory(plan_for(geom, SPEC), geom, X, c, SPEC, 3e-7, 100, "wide")


# ---------------------------------------------------------------- energy counts

@pytest.mark.parametrize("n_energy,n_it", [(33, 60), (336, 40), (337, 40)])
def test_energy_sum_paths_trajectory_parity(n_energy, n_it):
    pr = synth.problem("tiny")
    spec = spectral_with(n_energy)
    X, c = oracle_counts(pr.geom, spec, pr.f_true, pr.seed)
    assert_trajectory(plan_for(pr.geom, spec), pr.geom, X, c, spec, 3e-7, n_it, f"I={n_energy}")


# ---------------------------------------------------------------- batch

def test_batch_with_wide_and_vector_slots_bitwise():
    from paper_1801_06263_amd import Batch, Params
    tiny = synth.problem("tiny")
    scans = [(tiny.geom, tiny.spec, tiny.f_true), (WIDE, SPEC, synth.inserts_phantom(WIDE.n, 20.0)),
             (tiny.geom, spectral_with(337), tiny.f_true), (WIDE_OFFSET, spectral_with(340),
                                                             synth.random_phantom(30, 18.0, 4))]
    prm = Params(3e-7, "block", "clip", True)
    b = Batch(Params(1.0, "block", "clip", True), 6)
    bound = []
    for i, (geom, spec, f) in enumerate(scans):
        plan = plan_for(geom, spec)
        c = dev(sino(synth.poisson_counts(model.counts_model(pj.system_matrix(geom) @ f.reshape(3, -1).T, spec),
                                          40 + i), geom.n_views, geom.n_bins))
        st = plan.new_state(c)
        b.set_slot(i + 1, plan, st, prm.lam)
        bound.append((plan, c, st))
    b.iterate(5, use_graph=True)
    torch.cuda.synchronize()
    for i, (plan, c, st) in enumerate(bound):
        ref = plan.new_state(c)
        plan.mocca_iterate(ref, prm, 5)
        torch.cuda.synchronize()
        assert torch.equal(st.f, ref.f) and torch.equal(st.fbar, ref.fbar) and torch.equal(st.y, ref.y), i
        assert torch.isfinite(st.f).all()

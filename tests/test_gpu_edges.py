"""Edge cases of the GPU library: empty iteration counts, zero counts, rays
that miss the image, single-pixel / single-view / single-bin scans, one and
512 energies, a 2048^2 image, the largest image (4096^2) and ray count
(just under 2^27 rays) a plan accepts, and argument errors reported through
the C ABI."""
import ctypes
import warnings

import numpy as np
import pytest

import synth
from helpers import UPPER, dev, host, normwise
from oracle import model, mocca as omocca, projector as pj

warnings.filterwarnings("ignore", category=RuntimeWarning)
torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def plan_for(geom, spec):
    from paper_1801_06263_amd import Plan
    return Plan(geom, spec)


SPEC = synth.make_spectral(20, 119, 120.0, 1e5, e_step=5)


def test_zero_iterations_leave_state_unchanged():
    from paper_1801_06263_amd import Params
    geom = synth.make_geometry(24, 20.0, 12, 40)
    plan = plan_for(geom, SPEC)
    rng = np.random.default_rng(1)
    st = plan.new_state(dev(rng.uniform(10, 1e5, (4, 12, 40))), dev(rng.random((3, 24, 24))))
    f0, y0 = st.f.clone(), st.y.clone()
    plan.mocca_iterate(st, Params(1e-7), 0)
    assert torch.equal(st.f, f0) and torch.equal(st.y, y0)


def test_zero_counts_stay_finite():
    from paper_1801_06263_amd import Params
    geom = synth.make_geometry(24, 20.0, 12, 40)
    plan = plan_for(geom, SPEC)
    st = plan.new_state(torch.zeros(4, 12, 40, device="cuda"))
    for curv in ("clip", "window"):
        plan.mocca_iterate(st, Params(1e-7, "block", curv), 10)
        assert torch.isfinite(st.f).all() and torch.isfinite(st.y).all()
    d = float(plan.dtpl(st.f, st.c).item())
    assert np.isfinite(d) and d >= 0


def test_rays_missing_the_image_are_masked():
    from paper_1801_06263_amd import Params
    # a detector 3x wider than the fan needs: most rays miss the image
    geom = synth.make_geometry(32, 20.0, 16, 96, bin_cm=3 * synth.covering_bin_pitch(20.0, 50.0, 100.0, 96))
    plan = plan_for(geom, SPEC)
    rho = host(plan.ray_lengths()).ravel()
    ref = pj.square_chord(geom)
    assert (ref == 0).mean() > 0.5
    assert normwise(rho, ref) <= 1e-5
    rng = np.random.default_rng(3)
    st = plan.new_state(dev(rng.uniform(1e3, 1e5, (4, 16, 96))))
    plan.mocca_iterate(st, Params(3e-7), 5)
    y = host(st.y).reshape(4, -1)
    assert (y[:, rho == 0] == 0).all() and (np.abs(y[:, rho > 0]) > 0).any()


@pytest.mark.parametrize("n,views,bins", [(1, 1, 1), (1, 5, 3), (5, 1, 7), (3, 4, 1)])
def test_degenerate_scans(n, views, bins):
    geom = synth.make_geometry(n, 2.0, views, bins)
    plan = plan_for(geom, SPEC)
    X = pj.system_matrix(geom)
    rng = np.random.default_rng(n * 100 + views * 10 + bins)
    f = rng.random((3, n, n)).astype(np.float32)
    p = host(plan.forward_project(dev(f))).reshape(3, -1)
    ref = (X @ f.reshape(3, -1).astype(np.float64).T).T
    assert np.abs(p - ref).max() <= 1e-5 * max(np.abs(ref).max(), 1e-30)
    q = rng.random((3, views, bins)).astype(np.float32)
    b = host(plan.back_project(dev(q))).reshape(3, -1)
    refb = (X.T @ q.reshape(3, -1).astype(np.float64).T).T
    assert np.abs(b - refb).max() <= 1e-5 * max(np.abs(refb).max(), 1e-30)


@pytest.mark.parametrize("e_lo,e_hi,step", [(60, 60, 1), (20, 531, 1)])
def test_energy_counts_one_and_512(e_lo, e_hi, step):
    energies = np.arange(e_lo, e_hi + 1, step, dtype=float)
    mu = synth.attenuation_table(energies)
    s = np.full((4, energies.size), 1.0 / energies.size)
    spec = synth.Spectral(mu=mu, s=s, n0=np.full(4, 1e5))
    geom = synth.make_geometry(16, 20.0, 8, 32)
    plan = plan_for(geom, spec)
    rng = np.random.default_rng(energies.size)
    p = rng.random((256, 3)) * np.array([10.0, 1.0, 0.02])
    c = rng.uniform(1e3, 1e5, (256, 4))
    out = plan.spectral_model(dev(p.T.reshape(3, 8, 32)), dev(c.T.reshape(4, 8, 32)), fp64_small=True)
    p64 = p.astype(np.float32).astype(np.float64)
    chat = model.counts_model(p64, spec)
    assert normwise(host(out["chat"]).reshape(4, -1).T, chat) <= 1e-5
    A, B, g = model.matrices_AB(p64, spec)
    H = model.hessian_from_AB(A, B, g, c.astype(np.float32).astype(np.float64), spec)
    Hg = host(out["H"]).reshape(6, -1)
    for j, (m, n) in enumerate(UPPER):
        assert np.abs(Hg[j] - H[:, m, n]).max() <= 1e-4 * np.abs(H).max()


def test_large_image_sampled():
    """2048^2 image, 64 views x 2048 bins: forward and back-projection at sampled rays / pixels."""
    geom = synth.make_geometry(2048, 40.0, 64, 2048)
    plan = plan_for(geom, SPEC)
    f = synth.inserts_phantom(2048, 40.0, scale=2.0).astype(np.float32)
    p = host(plan.forward_project(dev(f))).reshape(3, 64, 2048)
    Xs = pj.system_matrix(geom, views=[0, 8, 31])
    ref = (Xs @ f.reshape(3, -1).astype(np.float64).T).T.reshape(3, 3, 2048)
    assert normwise(p[:, [0, 8, 31]], ref) <= 1e-5
    rng = np.random.default_rng(7)
    q = rng.random((1, 64, 2048)).astype(np.float32)
    b = host(plan.back_project(dev(q))).reshape(2048, 2048)
    for ix, iy in [(1024, 1024), (3, 1500), (2000, 17)]:
        col = pj.pixel_column(geom, ix, iy)
        refb = float(col @ q.ravel().astype(np.float64))
        assert abs(b[iy, ix] - refb) <= 1e-5 * abs(refb)


def test_maximum_image_sampled():
    """n = 4096, the largest image a plan accepts (32 views x 4096 bins): ray
    lengths against the closed-form chord of the image square, a forward
    projection at one view against the oracle, the back-projection at
    sampled pixels (corner and edge pixels included)."""
    n, V, D = 4096, 32, 4096
    geom = synth.make_geometry(n, 40.0, V, D)
    plan = plan_for(geom, SPEC)
    assert normwise(host(plan.ray_lengths()).ravel(), pj.square_chord(geom)) <= 1e-5
    rng = np.random.default_rng(8)
    f = rng.random((3, n, n), dtype=np.float32)
    p = host(plan.forward_project(dev(f))).reshape(3, V, D)
    Xs = pj.system_matrix(geom, views=[13])
    ref = (Xs @ f.reshape(3, -1).astype(np.float64).T).T
    assert normwise(p[:, 13], ref) <= 1e-5
    q = rng.random((1, V, D)).astype(np.float32)
    b = host(plan.back_project(dev(q))).reshape(n, n)
    pix = [(2048, 2048), (5, 3000), (4000, 77), (0, 0), (4095, 4095), (4095, 0), (1, 2048)]
    got = np.array([b[iy, ix] for ix, iy in pix])
    ref = np.array([pj.pixel_column(geom, ix, iy) @ q.ravel().astype(np.float64) for ix, iy in pix])
    assert normwise(got, ref) <= 1e-5, (got, ref)


def test_maximum_ray_count():
    """65535 views x 2048 bins, just under the plan's limit of 2^27 rays (a
    64^2 image whose 16 x 16 tiles shadow hundreds of bins): ray lengths and a
    forward projection at sampled views against the oracle, and adjointness
    <X f, q> = <f, X^T q> over every ray (FP64 dots of the FP32 results)."""
    n, V, D = 64, 65535, 2048
    geom = synth.make_geometry(n, 20.0, V, D)
    plan = plan_for(geom, SPEC)
    views = [0, 1, 32767, 65534]
    rho = plan.ray_lengths()
    assert normwise(host(rho[views]).ravel(), pj.square_chord(geom, views=views)) <= 1e-5
    del rho
    f = synth.inserts_phantom(n, 20.0).astype(np.float32)
    p = plan.forward_project(dev(f))
    Xs = pj.system_matrix(geom, views=views)
    ref = (Xs @ f.reshape(3, -1).astype(np.float64).T).T
    assert normwise(host(p[:, views]).reshape(3, -1), ref) <= 1e-5
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    q = torch.rand(1, V, D, device="cuda", generator=gen)
    b = plan.back_project(q)
    lhs = float((p[0].double() * q[0].double()).sum().item())
    rhs = float((dev(f[0]).double() * b[0].double()).sum().item())
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs), (lhs, rhs)


# ---------------------------------------------------------------- argument errors

def _c_plan(geom, spec):
    from paper_1801_06263_amd import osscir
    lib = osscir.load_library()
    g = osscir._Geometry(geom.n, geom.pixel_cm, geom.n_views, geom.n_bins, geom.sid_cm, geom.sdd_cm, geom.bin_cm,
                         geom.view0_rad, geom.arc_rad)
    mu = np.ascontiguousarray(spec.mu); s = np.ascontiguousarray(spec.s); n0 = np.ascontiguousarray(spec.n0)
    dp = ctypes.POINTER(ctypes.c_double)
    sp = osscir._Spectral(mu.shape[0], s.shape[0], s.shape[1], mu.ctypes.data_as(dp), s.ctypes.data_as(dp),
                          n0.ctypes.data_as(dp))
    h = ctypes.c_void_p()
    rc = lib.osscir_plan_create(ctypes.byref(g), ctypes.byref(sp), ctypes.byref(h))
    return lib, rc, h


def test_plan_argument_errors():
    geom = synth.make_geometry(16, 20.0, 8, 32)
    lib, rc, h = _c_plan(geom, SPEC)
    assert rc == 0
    lib.osscir_plan_destroy(h)
    bad_s = synth.Spectral(mu=SPEC.mu, s=SPEC.s * 1.01, n0=SPEC.n0)
    lib, rc, h = _c_plan(geom, bad_s)
    assert rc == -1 and b"sums to" in lib.osscir_last_error() and not h.value
    two_mat = synth.Spectral(mu=SPEC.mu[:2], s=SPEC.s, n0=SPEC.n0)
    lib, rc, _ = _c_plan(geom, two_mat)
    assert rc == -1 and b"n_mat=3" in lib.osscir_last_error()
    inside = synth.Geometry(n=16, pixel_cm=20 / 16, n_views=8, n_bins=32, sid_cm=5.0, sdd_cm=100.0, bin_cm=1.0)
    lib, rc, _ = _c_plan(inside, SPEC)
    assert rc == -1 and b"circumcircle" in lib.osscir_last_error()
    neg = synth.Spectral(mu=SPEC.mu, s=SPEC.s, n0=-SPEC.n0)
    lib, rc, _ = _c_plan(geom, neg)
    assert rc == -1


def test_iteration_argument_errors():
    from paper_1801_06263_amd import Params, osscir
    geom = synth.make_geometry(16, 20.0, 8, 32)
    plan = plan_for(geom, SPEC)
    st = plan.new_state(torch.ones(4, 8, 32, device="cuda"))
    with pytest.raises(osscir.OsscirError, match="lambda"):
        plan.mocca_iterate(st, Params(0.0), 1)
    small = osscir.State(st.f, st.fbar, st.y, st.c, st.work[:16])
    with pytest.raises(osscir.OsscirError, match="workspace"):
        plan.mocca_iterate(small, Params(1e-7), 1)
    with pytest.raises(osscir.OsscirError, match="n_ch"):
        lib = osscir.load_library()
        osscir._check(lib.osscir_forward_project(plan._h, ctypes.c_void_p(st.f.data_ptr()), 0,
                                                 ctypes.c_void_p(st.y.data_ptr()), None))
    with pytest.raises(ValueError):
        plan.forward_project(torch.ones(3, 15, 15, device="cuda"))

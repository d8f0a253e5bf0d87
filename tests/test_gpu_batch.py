"""Batched iterations (osscir_batch_*): every slot of a batch follows, bit for
bit, the trajectory the single-scan path (osscir_mocca_iterate) gives its scan
alone, whatever the other slots, the launch configuration, graph replay or
tuning; the single-scan path is in turn held to the FP64 oracle by
test_gpu_parity.py, and one slot here is compared with the oracle directly.

Bars: bit-exact (torch.equal) between batched and single-scan results; the
device's relative change of f within 1e-12 of the same quantity formed on the
host in FP64 from the single-scan iterates (only the summation order
differs); maps after 100 batched iterations within 1e-3 relative L2 of the
oracle.
"""
import math

import numpy as np
import pytest

import synth
from oracle import model, mocca as omocca, projector as pj

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def small_problems():
    """Four scans of different shapes (ragged tiles and workgroups, a half arc)."""
    spec5 = synth.make_spectral(20, 119, 120.0, 1e5, e_step=5)
    tiny = synth.problem("tiny")
    ragged = synth.Problem("ragged", synth.make_geometry(40, 20.0, 30, 100), spec5,
                           synth.inserts_phantom(40, 20.0), 11)
    offset = synth.Problem("offset", synth.Geometry(n=24, pixel_cm=0.7, n_views=17, n_bins=61, sid_cm=40.0,
                                                    sdd_cm=90.0, bin_cm=0.9, view0_rad=0.37, arc_rad=math.pi),
                           spec5, synth.random_phantom(24, 24 * 0.7, 12), 12)
    slice128 = synth.batch_slice(128, 0)
    return [tiny, ragged, offset, slice128]


LAM = {"tiny": 3e-7, "ragged": 3e-7, "offset": 3e-7}


def lam_of(pr):
    return LAM.get(pr.name, 2e-8)


def lib_counts(plan, pr):
    """Poisson counts at the phantom from the library's own counts model."""
    g = pr.geom
    p = plan.forward_project(dev(pr.f_true))
    chat = plan.spectral_model(p, torch.zeros(4, g.n_views, g.n_bins, device="cuda"))["chat"]
    return dev(synth.poisson_counts(host(chat), pr.seed))


@pytest.fixture(scope="module")
def scans():
    from paper_1801_06263_amd import Plan
    out = []
    for pr in small_problems():
        plan = Plan(pr.geom, pr.spec)
        out.append((pr, plan, lib_counts(plan, pr)))
    return out


def single_run(plan, c, params, n_iter):
    st = plan.new_state(c)
    plan.mocca_iterate(st, params, n_iter)
    torch.cuda.synchronize()
    return st


def same_state(a, b):
    return torch.equal(a.f, b.f) and torch.equal(a.fbar, b.fbar) and torch.equal(a.y, b.y)


def make_batch(scans, modes, max_slots=8, **cfg):
    from paper_1801_06263_amd import Batch
    b = Batch(modes, max_slots)
    if cfg:
        b.set_config(**cfg)
    states = []
    for i, (pr, plan, c) in enumerate(scans):
        st = plan.new_state(c)
        b.set_slot(i, plan, st, lam_of(pr))
        states.append(st)
    return b, states


@pytest.mark.parametrize("precond,curvature,fp64", [("block", "clip", True), ("block", "clip", False),
                                                    ("diag", "window", False)])
def test_batch_equals_single_bitwise(scans, precond, curvature, fp64):
    from paper_1801_06263_amd import Params
    from paper_1801_06263_amd.osscir import SLOT_RUNNING
    n_it = 7
    modes = Params(1.0, precond, curvature, fp64)
    b, states = make_batch(scans, modes)
    b.iterate(n_it, use_graph=True)
    status = b.status()
    for i, (pr, plan, c) in enumerate(scans):
        prm = Params(lam_of(pr), precond, curvature, fp64)
        ref_prev = single_run(plan, c, prm, n_it - 1)
        ref = single_run(plan, c, prm, n_it)
        assert same_state(states[i], ref), pr.name
        assert torch.isfinite(ref.f).all()
        state, iters, rel = status[i]
        assert state == SLOT_RUNNING and iters == n_it
        f1, f0 = host(ref.f), host(ref_prev.f)
        rel_ref = math.sqrt(((f1 - f0) ** 2).sum() / (f1 ** 2).sum())
        assert abs(rel - rel_ref) <= 1e-12 * rel_ref, (pr.name, rel, rel_ref)
    for i in range(len(scans), b.max_slots):
        assert status[i][0] == 0


def test_high_slot_indices(scans):
    """Slots 127..255 of a full-size batch (work-item codes with the top bit
    set) run the same trajectories as the single-scan path."""
    from paper_1801_06263_amd import Batch, Params
    from paper_1801_06263_amd.osscir import SLOT_RUNNING
    modes = Params(1.0, "block", "clip", True)
    b = Batch(modes, 256)
    slots = [255, 200, 128, 127]
    states = []
    for s, (pr, plan, c) in zip(slots, scans):
        st = plan.new_state(c)
        b.set_slot(s, plan, st, lam_of(pr))
        states.append(st)
    n_it = 4
    b.iterate(n_it, use_graph=True)
    status = b.status()
    for s, st, (pr, plan, c) in zip(slots, states, scans):
        assert status[s][:2] == (SLOT_RUNNING, n_it), (s, status[s])
        assert same_state(st, single_run(plan, c, Params(lam_of(pr), "block", "clip", True), n_it)), s
    assert all(status[i][0] == 0 for i in range(256) if i not in slots)


def test_graph_replays_match_eager(scans):
    """Graph replays against direct launches, one iteration at a time, with
    eager torch work and synchronisation between replays."""
    from paper_1801_06263_amd import Params
    modes = Params(1.0, "block", "clip", True)
    be, se = make_batch(scans, modes)
    bg, sg = make_batch(scans, modes)
    scratch = torch.randn(1 << 20, device="cuda")
    for it in range(5):
        be.iterate(1, use_graph=False)
        bg.iterate(1, use_graph=True)
        torch.cuda.synchronize()
        _ = float((scratch * it).sum())
        for a, g in zip(se, sg):
            assert same_state(a, g), it
    assert be.status() == bg.status()


def test_launch_configuration_does_not_change_results(scans):
    from paper_1801_06263_amd import Params
    modes = Params(1.0, "block", "clip", True)
    cfgs = [dict(fp_rays=64, fp_wgs=8, fp_xcd=0, spec_rays=64, spec_wgs=16, spec_xcd=0, bp_wgs=8, bp_xcd=0),
            dict(fp_rays=128, fp_wgs=4096, fp_xcd=1, spec_rays=256, spec_wgs=65536, spec_xcd=1, bp_wgs=16384,
                 bp_xcd=1)]
    outs = []
    for cfg in cfgs:
        b, states = make_batch(scans, modes, **cfg)
        assert b.get_config() == cfg
        b.iterate(4, use_graph=True)
        torch.cuda.synchronize()
        outs.append(states)
    for a, g in zip(*outs):
        assert same_state(a, g)


def test_stopping_rules(scans):
    from paper_1801_06263_amd import Batch, Params
    from paper_1801_06263_amd.osscir import SLOT_DONE, SLOT_RUNNING
    pr, plan, c = scans[0]
    prm = Params(lam_of(pr), "block", "clip", True)
    # host relative changes of the single-scan trajectory
    st = plan.new_state(c)
    rels, prev = [], host(st.f)
    for _ in range(10):
        plan.mocca_iterate(st, prm, 1)
        cur = host(st.f)
        rels.append(math.sqrt(((cur - prev) ** 2).sum() / (cur ** 2).sum()))
        prev = cur
    k = next(n for n in range(3, 10) if rels[n] < 0.99 * min(rels[:n]))
    tol = math.sqrt(rels[k] * min(rels[:k]))  # first reached at iteration k + 1
    b = Batch(Params(1.0, "block", "clip", True), 4)
    sa, sb, sc = plan.new_state(c), plan.new_state(c), plan.new_state(c)
    b.set_slot(0, plan, sa, prm.lam, max_iter=3)
    b.set_slot(1, plan, sb, prm.lam)
    b.set_slot(2, plan, sc, prm.lam, tol=tol)
    b.iterate(12)
    status = b.status()
    assert status[0][:2] == (SLOT_DONE, 3)
    assert status[1][:2] == (SLOT_RUNNING, 12)
    assert status[2][:2] == (SLOT_DONE, k + 1)
    assert same_state(sa, single_run(plan, c, prm, 3))
    assert same_state(sb, single_run(plan, c, prm, 12))
    assert same_state(sc, single_run(plan, c, prm, k + 1))


def test_rebind_and_clear(scans):
    from paper_1801_06263_amd import Batch, Params
    (pa, plan_a, ca), (pb, plan_b, cb), (pc, plan_c, cc) = scans[:3]
    modes = Params(1.0, "block", "clip", True)
    b = Batch(modes, 3)
    sa, sb = plan_a.new_state(ca), plan_b.new_state(cb)
    b.set_slot(0, plan_a, sa, lam_of(pa))
    b.set_slot(1, plan_b, sb, lam_of(pb))
    b.iterate(3)
    b.clear_slot(1)
    sc = plan_c.new_state(cc)
    b.set_slot(2, plan_c, sc, lam_of(pc))
    b.iterate(3)
    status = b.status()
    assert status[0][1] == 6 and status[1][0] == 0 and status[2][1] == 3
    prm = lambda pr: Params(lam_of(pr), "block", "clip", True)
    assert same_state(sa, single_run(plan_a, ca, prm(pa), 6))
    assert same_state(sb, single_run(plan_b, cb, prm(pb), 3))
    assert same_state(sc, single_run(plan_c, cc, prm(pc), 3))
    # rebinding slot 0 restarts it on the new state
    sa2 = plan_a.new_state(ca)
    b.set_slot(0, plan_a, sa2, lam_of(pa))
    b.iterate(2)
    assert b.status()[0][1] == 2
    assert same_state(sa2, single_run(plan_a, ca, prm(pa), 2))


def test_tuner_leaves_trajectories_unchanged(scans):
    from paper_1801_06263_amd import Params
    modes = Params(1.0, "block", "clip", True)
    b, states = make_batch(scans, modes)
    b.iterate(3)
    cfg = b.tune(1)
    assert cfg == b.get_config()
    assert cfg["fp_rays"] in (64, 128, 256) and cfg["bp_wgs"] % 8 == 0
    assert [s[1] for s in b.status()[:len(scans)]] == [3] * len(scans)
    b.iterate(3)
    for (pr, plan, c), st in zip(scans, states):
        assert same_state(st, single_run(plan, c, Params(lam_of(pr), "block", "clip", True), 6)), pr.name


def test_split_back_projection_scans_in_a_batch_with_slot_workspaces(scans):
    """Scans of few 16 x 16 tiles split their single-scan back-projection
    over views (per-part FP64 sums in the workspace, added in order); a batch
    slot forms the same sums in registers, so it needs the smaller workspace
    osscir_batch_workspace_bytes and still equals the scan run alone."""
    from paper_1801_06263_amd import Batch, Params
    from paper_1801_06263_amd.osscir import OsscirError
    n_it = 9
    modes = Params(1.0, "block", "clip", True)
    b = Batch(modes, 4)
    states = []
    for i, (pr, plan, c) in enumerate(scans):
        assert plan.batch_workspace_bytes <= plan.workspace_bytes
        st = plan.new_state(c, batch=True)
        b.set_slot(i, plan, st, lam_of(pr))
        states.append(st)
    assert any(plan.batch_workspace_bytes < plan.workspace_bytes for _, plan, _ in scans)  # some scan splits
    b.iterate(n_it)
    for i, (pr, plan, c) in enumerate(scans):
        ref = single_run(plan, c, Params(lam_of(pr), "block", "clip", True), n_it)
        assert same_state(states[i], ref), pr.name
    # a workspace one byte short of a slot's is refused
    pr, plan, c = scans[0]
    st = plan.new_state(c, batch=True)
    st.work = st.work[:plan.batch_workspace_bytes - 1]
    with pytest.raises(OsscirError, match="workspace"):
        b.set_slot(0, plan, st, lam_of(pr))


def test_slot_with_non_finite_counts_fails_alone(scans):
    """A slot whose counts hold a NaN (on a ray through the image) stops with
    SLOT_FAILED after its first iteration, its maps no longer finite; the
    other slot runs on and still equals its scan run alone."""
    from paper_1801_06263_amd import Batch, Params
    from paper_1801_06263_amd.osscir import SLOT_FAILED, SLOT_RUNNING
    (pr0, plan0, c0), (pr1, plan1, c1) = scans[0], scans[1]
    bad = c0.clone()
    bad[0, 0, bad.shape[2] // 2] = float("nan")  # view 0's central bin
    b = Batch(Params(1.0, "block", "clip", True), 2)
    s0, s1 = plan0.new_state(bad), plan1.new_state(c1)
    b.set_slot(0, plan0, s0, lam_of(pr0), tol=1e-12)
    b.set_slot(1, plan1, s1, lam_of(pr1))
    b.iterate(5)
    status = b.status()
    assert status[0][:2] == (SLOT_FAILED, 1), status[0]
    assert not torch.isfinite(s0.f).all()
    assert status[1][:2] == (SLOT_RUNNING, 5), status[1]
    assert same_state(s1, single_run(plan1, c1, Params(lam_of(pr1), "block", "clip", True), 5))


def test_batched_slot_matches_oracle():
    """The tiny scan run inside a batch (beside a 128^2 slice) for 100
    iterations against the FP64 oracle's trajectory."""
    from paper_1801_06263_amd import Batch, Params, Plan
    pr = synth.problem("tiny")
    X = pj.system_matrix(pr.geom)
    c = synth.poisson_counts(model.counts_model(X @ pr.f_true.reshape(3, -1).T, pr.spec), pr.seed)
    lam, n_it = 3e-7, 100
    ref, _ = omocca.mocca(X, c, pr.spec, lam, n_it, "block", "clip")
    plan = Plan(pr.geom, pr.spec)
    other = synth.batch_slice(128, 5)
    plan_o = Plan(other.geom, other.spec)
    g = pr.geom
    st = plan.new_state(dev(np.ascontiguousarray(c.T.reshape(4, g.n_views, g.n_bins))))
    so = plan_o.new_state(lib_counts(plan_o, other))
    b = Batch(Params(1.0, "block", "clip", True), 2)
    b.set_slot(1, plan, st, lam)
    b.set_slot(0, plan_o, so, 2e-8)
    b.iterate(n_it)
    f = host(st.f).reshape(3, -1)
    for m in range(3):
        rel = np.linalg.norm(f[m] - ref.f[m]) / np.linalg.norm(ref.f[m])
        print(f"material {m}: rel L2 {rel:.2e}")
        assert rel <= 1e-3


def test_full_mix_bitwise_in_tuned_configuration():
    """The 24-slice mix (128^2 .. 512^2) in the tuned launch configuration:
    every slot equals its scan run alone."""
    from paper_1801_06263_amd import Batch, Params, Plan
    mix = synth.batch_mix(6)
    plans = {}
    modes = Params(1.0, "block", "clip", True)
    b = Batch(modes, len(mix))
    items = []
    for i, pr in enumerate(mix):
        n = pr.geom.n
        if n not in plans:
            plans[n] = Plan(pr.geom, pr.spec)
        c = lib_counts(plans[n], pr)
        st = plans[n].new_state(c)
        b.set_slot(i, plans[n], st, 2e-8)
        items.append((pr, c, st))
    b.iterate(1)
    b.tune(1)
    b.iterate(2)
    torch.cuda.synchronize()
    for pr, c, st in items:
        ref = single_run(plans[pr.geom.n], c, Params(2e-8, "block", "clip", True), 3)
        assert same_state(st, ref), pr.name
        assert torch.isfinite(st.f).all()


def test_batch_argument_errors(scans):
    from paper_1801_06263_amd import Batch, Params
    from paper_1801_06263_amd.osscir import OsscirError
    pr, plan, c = scans[0]
    with pytest.raises(OsscirError):
        Batch(Params(1.0), 0)
    with pytest.raises(OsscirError):
        Batch(Params(1.0), 257)
    b = Batch(Params(1.0), 2)
    st = plan.new_state(c)
    with pytest.raises(OsscirError):
        b.set_slot(2, plan, st, 1e-7)
    with pytest.raises(OsscirError):
        b.set_slot(0, plan, st, 0.0)
    with pytest.raises(OsscirError):
        b.set_slot(0, plan, st, 1e-7, max_iter=-1)
    small = plan.new_state(c)
    small.work = small.work[:16]
    with pytest.raises(OsscirError):
        b.set_slot(0, plan, small, 1e-7)
    with pytest.raises(OsscirError):
        b.set_config(fp_rays=96)
    with pytest.raises(OsscirError):
        b.set_config(bp_wgs=12)
    with pytest.raises(OsscirError):
        b.clear_slot(-1)
    b.iterate(3)  # nothing bound: a no-op
    assert all(s[0] == 0 for s in b.status())


# ---------------------------------------------------------------- nested loops in a batch

def nested_run(plan, c, params, chunks):
    """osscir_mocca_iterate_nested called once per (n_outer, n_inner) chunk,
    on one state and one p0 buffer."""
    st = plan.new_state(c)
    p0 = None
    for n_outer, n_inner in chunks:
        p0, _ = plan.mocca_iterate_nested(st, params, n_outer, n_inner, p0=p0)
    torch.cuda.synchronize()
    return st


@pytest.mark.parametrize("precond,curvature", [("block", "clip"), ("diag", "window")])
@pytest.mark.parametrize("use_graph", [True, False])
def test_nested_slots_equal_single_scan_nested(scans, precond, curvature, use_graph):
    """Slots with 2 and 3 inner steps per expansion point beside single-loop
    slots: each follows osscir_mocca_iterate_nested (or the single loop) bit
    for bit; iters counts inner steps."""
    from paper_1801_06263_amd import Batch, Params
    modes = Params(1.0, precond, curvature, True)
    b = Batch(modes, 8)
    inner = [2, 3, 1, 2]
    states = []
    for i, ((pr, plan, c), k) in enumerate(zip(scans, inner)):
        st = plan.new_state(c)
        b.set_slot(i, plan, st, lam_of(pr), n_inner=k)
        states.append(st)
    n_it = 6
    b.iterate(n_it, use_graph=use_graph)
    status = b.status()
    for i, ((pr, plan, c), k) in enumerate(zip(scans, inner)):
        prm = Params(lam_of(pr), precond, curvature, True)
        ref = nested_run(plan, c, prm, [(n_it // k, k)])
        assert same_state(states[i], ref), (pr.name, k)
        assert status[i][1] == n_it


def test_nested_slot_stops_inside_an_outer_iteration(scans):
    """max_iter = 6 with 4 inner steps: one whole outer iteration and the first
    two steps of the next, as the single-scan calls (1 x 4) then (1 x 2)."""
    from paper_1801_06263_amd import Batch, Params
    from paper_1801_06263_amd.osscir import SLOT_DONE
    pr, plan, c = scans[0]
    modes = Params(1.0, "block", "clip", True)
    b = Batch(modes, 4)
    st = plan.new_state(c)
    b.set_slot(0, plan, st, lam_of(pr), max_iter=6, n_inner=4)
    b.iterate(9, use_graph=True)
    assert b.status()[0][:2] == (SLOT_DONE, 6)
    ref = nested_run(plan, c, Params(lam_of(pr), "block", "clip", True), [(1, 4), (1, 2)])
    assert same_state(st, ref)


def test_nesting_change_recaptures_and_tuning_keeps_p0(scans):
    """Single-loop slots first (graph without the nested kernel variant), then a
    nested slot bound between replays; tuning in the middle restores every
    slot, p0 included."""
    from paper_1801_06263_amd import Batch, Params
    modes = Params(1.0, "block", "clip", True)
    b = Batch(modes, 4)
    (pr0, plan0, c0), (pr1, plan1, c1) = scans[0], scans[1]
    s0 = plan0.new_state(c0)
    b.set_slot(0, plan0, s0, lam_of(pr0))
    b.iterate(2, use_graph=True)
    s1 = plan1.new_state(c1)
    b.set_slot(1, plan1, s1, lam_of(pr1), n_inner=3)
    b.iterate(4, use_graph=True)
    b.tune(1)
    b.iterate(2, use_graph=True)
    prm0 = Params(lam_of(pr0), "block", "clip", True)
    prm1 = Params(lam_of(pr1), "block", "clip", True)
    assert same_state(s0, single_run(plan0, c0, prm0, 8))
    assert same_state(s1, nested_run(plan1, c1, prm1, [(2, 3)]))


def test_nested_slot_argument_errors(scans):
    from paper_1801_06263_amd import Batch, Params
    from paper_1801_06263_amd.osscir import OsscirError, _lib, _stream_handle
    import ctypes
    pr, plan, c = scans[0]
    b = Batch(Params(1.0), 2)
    st = plan.new_state(c)
    with pytest.raises(OsscirError, match="n_inner"):
        b.set_slot(0, plan, st, lam_of(pr), n_inner=0)
    cst = plan._c_state(st)
    rc = _lib.osscir_batch_set_slot_nested(b._h, 0, plan._h, ctypes.byref(cst), 1e-7, 0, 0.0, 3, None,
                                           _stream_handle(None))
    assert rc == -1


def test_nested_slot_with_per_bin_spectra(scans):
    """A nested slot whose scan has one response per detector bin (the per-bin
    call of the batched kernel's nested variant) beside a single-loop slot."""
    from paper_1801_06263_amd import Batch, Params, Plan
    pr = synth.problem("tiny")
    det = synth.make_detector_spectral(pr.geom.n_bins, 20, 119, 120.0, 1e5, 77)
    plan = Plan(pr.geom, det)
    c = lib_counts(plan, pr)
    modes = Params(1.0, "block", "clip", True)
    b = Batch(modes, 4)
    st = plan.new_state(c)
    b.set_slot(0, plan, st, 1e-6, n_inner=3)
    pr1, plan1, c1 = scans[1]
    s1 = plan1.new_state(c1)
    b.set_slot(1, plan1, s1, lam_of(pr1))
    b.iterate(6, use_graph=True)
    assert same_state(st, nested_run(plan, c, Params(1e-6, "block", "clip", True), [(2, 3)]))
    assert same_state(s1, single_run(plan1, c1, Params(lam_of(pr1), "block", "clip", True), 6))

"""osscir_mocca_iterate_noalloc (the iteration with the library's static
scratch as workspace) against osscir_mocca_iterate on the same inputs: bit
for bit, on two calls in a row (the second on a smaller scan), with and
without the per-iteration D_TPL, and the size limit."""
import ctypes

import numpy as np
import pytest

import synth
from helpers import dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def scan(n, views, bins, e_step, seed):
    from paper_1801_06263_amd import Plan
    geom = synth.make_geometry(n, 20.0, views, bins)
    spec = synth.make_spectral(20, 119, 120.0, 1e5, e_step=e_step)
    plan = Plan(geom, spec)
    p = plan.forward_project(dev(synth.inserts_phantom(n, 20.0)))
    chat = plan.spectral_model(p, torch.zeros(4, views, bins, device="cuda"))["chat"]
    torch.cuda.synchronize()
    c = dev(synth.poisson_counts(chat.double().cpu().numpy(), seed))
    return plan, c


def same(a, b):
    return torch.equal(a.f, b.f) and torch.equal(a.fbar, b.fbar) and torch.equal(a.y, b.y)


def test_noalloc_equals_workspace_path_on_two_calls():
    from paper_1801_06263_amd import Params
    params = Params(3e-7, "block", "clip", True)
    big, c_big = scan(64, 64, 128, 1, 5)
    small, c_small = scan(40, 30, 100, 1, 6)
    for plan, c, n_it, with_dtpl in ((big, c_big, 12, True), (small, c_small, 9, False)):
        ref = plan.new_state(c)
        d_ref = plan.mocca_iterate(ref, params, n_it, dtpl=with_dtpl)
        st = plan.new_state(c)
        d = torch.empty(n_it, dtype=torch.float64, device="cuda") if with_dtpl else None
        plan.mocca_iterate_noalloc(st, params, n_it, dtpl=d)
        torch.cuda.synchronize()
        assert same(st, ref)
        assert torch.isfinite(st.f).all()
        if with_dtpl:
            assert torch.equal(d, d_ref)
    # a third call on the first scan again, after the smaller one used the scratch
    ref = big.new_state(c_big)
    big.mocca_iterate(ref, params, 5)
    st = big.new_state(c_big)
    big.mocca_iterate_noalloc(st, params, 5)
    torch.cuda.synchronize()
    assert same(st, ref)


def test_noalloc_rejects_scans_beyond_the_static_scratch():
    from paper_1801_06263_amd import Params, Plan
    from paper_1801_06263_amd.osscir import OsscirError
    geom = synth.make_geometry(512, 40.0, 1440, 1024)
    plan = Plan(geom, synth.make_spectral(20, 119, 120.0, 1e5, e_step=20))
    assert plan.workspace_bytes > (64 << 20)
    c = torch.zeros(4, 1440, 1024, device="cuda")
    st = plan.new_state(c)
    with pytest.raises(OsscirError, match="static"):
        plan.mocca_iterate_noalloc(st, Params(3e-7, "block", "clip", True), 1)

"""Thin ctypes binding of libosscir (include/osscir.h).

Argument marshalling only: every step of the reconstruction runs in the HIP
library.  PyTorch supplies device memory and the current stream.  If the
shared library has not been built this module raises on first use; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libosscir.so")

PRECOND_DIAG, PRECOND_BLOCK = 0, 1
CURV_WINDOW, CURV_CLIP = 0, 1

c_int32, c_double, c_size_t, c_void_p = ctypes.c_int32, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


class _Geometry(ctypes.Structure):
    _fields_ = [("n", c_int32), ("pixel_cm", c_double), ("n_views", c_int32), ("n_bins", c_int32),
                ("sid_cm", c_double), ("sdd_cm", c_double), ("bin_cm", c_double),
                ("view0_rad", c_double), ("arc_rad", c_double)]


class _Spectral(ctypes.Structure):
    _fields_ = [("n_mat", c_int32), ("n_win", c_int32), ("n_energy", c_int32),
                ("mu", _dp), ("s", _dp), ("n0", _dp), ("n_resp", c_int32), ("n0_ray", _dp)]


class _Params(ctypes.Structure):
    _fields_ = [("lam", c_double), ("precond", c_int32), ("curvature", c_int32), ("fp64_small", c_int32)]


class _State(ctypes.Structure):
    _fields_ = [("f", c_void_p), ("fbar", c_void_p), ("y", c_void_p), ("c", c_void_p),
                ("work", c_void_p), ("work_bytes", c_size_t)]


class _SlotStatus(ctypes.Structure):
    _fields_ = [("state", c_int32), ("iters", c_int32), ("rel_change", c_double)]


class _BatchConfig(ctypes.Structure):
    _fields_ = [("fp_rays", c_int32), ("fp_wgs", c_int32), ("fp_xcd", c_int32),
                ("spec_rays", c_int32), ("spec_wgs", c_int32), ("spec_xcd", c_int32),
                ("bp_wgs", c_int32), ("bp_xcd", c_int32)]


SLOT_EMPTY, SLOT_RUNNING, SLOT_DONE, SLOT_FAILED = 0, 1, 2, 3

# name -> (restype, argtypes) for every entry point of include/osscir.h
SIGNATURES = {
    "osscir_plan_create": (c_int32, [ctypes.POINTER(_Geometry), ctypes.POINTER(_Spectral), ctypes.POINTER(c_void_p)]),
    "osscir_plan_destroy": (c_int32, [c_void_p]),
    "osscir_plan_set_energy_sums": (c_int32, [c_void_p, c_int32]),
    "osscir_workspace_bytes": (c_int32, [c_void_p, ctypes.POINTER(c_size_t)]),
    "osscir_batch_workspace_bytes": (c_int32, [c_void_p, ctypes.POINTER(c_size_t)]),
    "osscir_ray_lengths": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "osscir_ray_table": (c_int32, [ctypes.POINTER(_Geometry), _dp, _dp]),
    "osscir_forward_project": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "osscir_back_project": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "osscir_spectral_model": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_int32, c_void_p]),
    "osscir_block_spc_steps": (c_int32, [c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p, c_size_t,
                                         c_void_p]),
    "osscir_diag_spc_steps": (c_int32, [c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p, c_size_t,
                                        c_void_p]),
    "osscir_mocca_iterate": (c_int32, [c_void_p, ctypes.POINTER(_Params), ctypes.POINTER(_State), c_int32, c_void_p,
                                       c_void_p]),
    "osscir_mocca_iterate_nested": (c_int32, [c_void_p, ctypes.POINTER(_Params), ctypes.POINTER(_State), c_int32,
                                              c_int32, c_void_p, c_void_p, c_void_p]),
    "osscir_mocca_stage": (c_int32, [c_void_p, ctypes.POINTER(_Params), ctypes.POINTER(_State), c_int32, c_void_p]),
    "osscir_mocca_iterate_noalloc": (c_int32, [c_void_p, ctypes.POINTER(_Params), c_void_p, c_void_p, c_void_p,
                                               c_void_p, c_int32, c_void_p, c_void_p]),
    "osscir_ray_nnz": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "osscir_dtpl": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "osscir_mu_pc_basis": (c_int32, [ctypes.POINTER(_Spectral), _dp, _dp]),
    "osscir_material_transform": (c_int32, [_dp, c_void_p, c_void_p, c_int32, c_void_p]),
    "osscir_batch_create": (c_int32, [ctypes.POINTER(_Params), c_int32, ctypes.POINTER(c_void_p)]),
    "osscir_batch_destroy": (c_int32, [c_void_p]),
    "osscir_batch_set_slot_nested": (c_int32, [c_void_p, c_int32, c_void_p, ctypes.POINTER(_State), c_double,
                                               c_int32, c_double, c_int32, c_void_p, c_void_p]),
    "osscir_batch_set_slot": (c_int32, [c_void_p, c_int32, c_void_p, ctypes.POINTER(_State), c_double, c_int32,
                                        c_double, c_void_p]),
    "osscir_batch_clear_slot": (c_int32, [c_void_p, c_int32]),
    "osscir_batch_iterate": (c_int32, [c_void_p, c_int32, c_int32, c_void_p]),
    "osscir_batch_status": (c_int32, [c_void_p, ctypes.POINTER(_SlotStatus), c_void_p]),
    "osscir_batch_get_config": (c_int32, [c_void_p, ctypes.POINTER(_BatchConfig)]),
    "osscir_batch_set_config": (c_int32, [c_void_p, ctypes.POINTER(_BatchConfig)]),
    "osscir_batch_tune": (c_int32, [c_void_p, c_int32, ctypes.POINTER(_BatchConfig), c_void_p]),
    "osscir_last_error": (ctypes.c_char_p, []),
    "osscir_version": (ctypes.c_char_p, []),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libosscir.so and declare its signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libosscir.so not built at {path}: run `python -m paper_1801_06263_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class OsscirError(RuntimeError):
    pass


def _check(rc: int):
    if rc != 0:
        msg = _lib.osscir_last_error().decode(errors="replace")
        raise OsscirError(f"osscir error {rc}: {msg}")


def _stream_handle(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return c_void_p(s.cuda_stream)


def _dev(t, shape=None, dtype=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return c_void_p(t.data_ptr())


@dataclasses.dataclass
class Params:
    lam: float
    precond: str = "block"       # "block" | "diag"
    curvature: str = "clip"      # "clip" | "window"
    fp64_small: bool = False     # per-ray 3x3 / 4x4 tail in FP64 (FP32 meets the 1e-3 map bar)

    def to_c(self) -> _Params:
        pre = {"diag": PRECOND_DIAG, "block": PRECOND_BLOCK}[self.precond]
        cur = {"window": CURV_WINDOW, "clip": CURV_CLIP}[self.curvature]
        return _Params(float(self.lam), pre, cur, int(bool(self.fp64_small)))


@dataclasses.dataclass
class State:
    """Device-resident iteration state (torch CUDA tensors)."""
    f: "object"      # [3, n, n] f32
    fbar: "object"   # [3, n, n] f32
    y: "object"      # [4, V, D] f32
    c: "object"      # [4, V, D] f32
    work: "object"   # [workspace_bytes] u8


class Plan:
    """A scan (geometry + spectral tables) prepared on the current device."""

    def __init__(self, geom, spec):
        lib = load_library()
        self.n, self.n_views, self.n_bins = int(geom.n), int(geom.n_views), int(geom.n_bins)
        g = _c_geometry(geom)
        self._mu = np.ascontiguousarray(spec.mu, dtype=np.float64)
        self._s = np.ascontiguousarray(spec.s, dtype=np.float64)
        # s [W, I] shared by every ray, or [D, W, I] per detector bin; incident
        # counts n0 [W] or [D, W], and optionally per ray: n0_ray [V, D, W]
        n0_ray = getattr(spec, "n0_ray", None)
        self._n0 = np.ascontiguousarray(spec.n0_nominal if n0_ray is not None else spec.n0, dtype=np.float64)
        self._n0_ray = None
        if n0_ray is not None:
            self._n0_ray = np.ascontiguousarray(n0_ray, dtype=np.float64).reshape(self.n_views, self.n_bins, -1)
        n_resp = self._s.shape[0] if self._s.ndim == 3 else 1
        self.per_bin = self._s.ndim == 3
        sp = _Spectral(self._mu.shape[0], self._s.shape[-2], self._s.shape[-1],
                       self._mu.ctypes.data_as(_dp), self._s.ctypes.data_as(_dp), self._n0.ctypes.data_as(_dp),
                       n_resp, self._n0_ray.ctypes.data_as(_dp) if self._n0_ray is not None else None)
        h = c_void_p()
        _check(lib.osscir_plan_create(ctypes.byref(g), ctypes.byref(sp), ctypes.byref(h)))
        self._h = h
        nb = c_size_t()
        _check(lib.osscir_workspace_bytes(self._h, ctypes.byref(nb)))
        self.workspace_bytes = int(nb.value)
        _check(lib.osscir_batch_workspace_bytes(self._h, ctypes.byref(nb)))
        self.batch_workspace_bytes = int(nb.value)  # a batch slot's (at most workspace_bytes)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(_lib.osscir_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_energy_sums(self, matrix_cores: bool):
        """Energy sums of the spectral step on the matrix cores (True, the
        default where it applies) or as per-ray vector FMAs (False)."""
        _check(_lib.osscir_plan_set_energy_sums(self._h, int(bool(matrix_cores))))

    # -- shapes
    @property
    def sino_shape(self):
        return (self.n_views, self.n_bins)

    @property
    def img_shape(self):
        return (self.n, self.n)

    def _empty(self, *shape, dtype=None):
        import torch
        return torch.empty(*shape, dtype=dtype or torch.float32, device="cuda")

    def workspace(self, batch: bool = False):
        import torch
        return torch.empty(self.batch_workspace_bytes if batch else self.workspace_bytes, dtype=torch.uint8,
                           device="cuda")

    # -- entry points
    def ray_lengths(self, stream=None):
        out = self._empty(*self.sino_shape)
        _check(_lib.osscir_ray_lengths(self._h, _dev(out), _stream_handle(stream)))
        return out

    def forward_project(self, f, out=None, stream=None):
        import torch
        nch = f.shape[0]
        fp = _dev(f, (nch, self.n, self.n), torch.float32, "f")
        out = self._empty(nch, *self.sino_shape) if out is None else out
        _check(_lib.osscir_forward_project(self._h, fp, nch, _dev(out, (nch, *self.sino_shape), torch.float32, "p"),
                                           _stream_handle(stream)))
        return out

    def back_project(self, q, out=None, stream=None):
        import torch
        nch = q.shape[0]
        qp = _dev(q, (nch, *self.sino_shape), torch.float32, "q")
        out = self._empty(nch, self.n, self.n) if out is None else out
        _check(_lib.osscir_back_project(self._h, qp, nch, _dev(out, (nch, self.n, self.n), torch.float32, "b"),
                                        _stream_handle(stream)))
        return out

    def spectral_model(self, p, c, fp64_small=False, stream=None):
        import torch
        V, D = self.sino_shape
        out = {"chat": self._empty(4, V, D), "r": self._empty(4, V, D), "G": self._empty(12, V, D),
               "H": self._empty(6, V, D), "Hplus": self._empty(6, V, D)}
        _check(_lib.osscir_spectral_model(
            self._h, _dev(p, (3, V, D), torch.float32, "p"), _dev(c, (4, V, D), torch.float32, "c"),
            _dev(out["chat"]), _dev(out["r"]), _dev(out["G"]), _dev(out["H"]), _dev(out["Hplus"]),
            int(bool(fp64_small)), _stream_handle(stream)))
        return out

    def spc_steps(self, G, lam, precond="block", work=None, stream=None):
        import torch
        V, D = self.sino_shape
        work = self.workspace() if work is None else work
        sigma = self._empty(4, V, D)
        img = self._empty(6 if precond == "block" else 3, self.n, self.n)
        fn = _lib.osscir_block_spc_steps if precond == "block" else _lib.osscir_diag_spc_steps
        _check(fn(self._h, _dev(G, (12, V, D), torch.float32, "G"), float(lam), _dev(sigma), _dev(img),
                  _dev(work), work.numel(), _stream_handle(stream)))
        return sigma, img

    def new_state(self, c, f0=None, batch: bool = False):
        """Device state for MOCCA from counts c [4, V, D] (a tensor or a host
        array; f0 = fbar0 = f0 or 0, y0 = 0).  batch: with the smaller
        workspace of a batch slot (then for batch slots only)."""
        import torch
        f = torch.zeros(3, self.n, self.n, dtype=torch.float32, device="cuda") if f0 is None \
            else f0.to(device="cuda", dtype=torch.float32).contiguous().clone()
        c = torch.as_tensor(np.ascontiguousarray(c, dtype=np.float32)) if isinstance(c, np.ndarray) else c
        return State(f=f, fbar=f.clone(), y=torch.zeros(4, *self.sino_shape, dtype=torch.float32, device="cuda"),
                     c=c.to(device="cuda", dtype=torch.float32).contiguous(), work=self.workspace(batch))

    def _c_state(self, state: State) -> _State:
        import torch
        V, D = self.sino_shape
        return _State(_dev(state.f, (3, self.n, self.n), torch.float32, "f").value,
                      _dev(state.fbar, (3, self.n, self.n), torch.float32, "fbar").value,
                      _dev(state.y, (4, V, D), torch.float32, "y").value,
                      _dev(state.c, (4, V, D), torch.float32, "c").value,
                      _dev(state.work, None, torch.uint8, "work").value, state.work.numel())

    def mocca_iterate(self, state: State, params: Params, n_iter: int, dtpl: bool = False, stream=None):
        """Run n_iter iterations in place; returns a [n_iter] float64 device tensor of D_TPL if asked."""
        import torch
        st = self._c_state(state)
        out = torch.empty(max(n_iter, 1), dtype=torch.float64, device="cuda") if dtpl else None
        prm = params.to_c()
        _check(_lib.osscir_mocca_iterate(self._h, ctypes.byref(prm), ctypes.byref(st), int(n_iter),
                                         _dev(out) if dtpl else None, _stream_handle(stream)))
        return out

    def mocca_iterate_nested(self, state: State, params: Params, n_outer: int, n_inner: int, p0=None,
                             dtpl: bool = False, stream=None):
        """Nested loops in place: n_outer expansion points (f0 = fbar at each
        outer start), n_inner CPPD steps on the quadratic at each.  p0: an
        optional [3, V, D] float32 device tensor for X f0 (allocated if None;
        returned).  Returns (p0, D_TPL [n_outer * n_inner] float64 or None)."""
        import torch
        V, D = self.sino_shape
        if p0 is None:
            p0 = torch.empty((3, V, D), dtype=torch.float32, device="cuda")
        st = self._c_state(state)
        total = max(int(n_outer) * int(n_inner), 1)
        out = torch.empty(total, dtype=torch.float64, device="cuda") if dtpl else None
        prm = params.to_c()
        _check(_lib.osscir_mocca_iterate_nested(self._h, ctypes.byref(prm), ctypes.byref(st), int(n_outer),
                                                int(n_inner), _dev(p0, (3, V, D), torch.float32, "p0"),
                                                _dev(out) if dtpl else None, _stream_handle(stream)))
        return p0, out

    def mocca_iterate_noalloc(self, state: State, params: Params, n_iter: int, dtpl=None, stream=None):
        """As mocca_iterate, with the library's static scratch in place of
        state.work (which is not touched); dtpl: an optional [n_iter]
        float64 device tensor the caller allocated."""
        import torch
        V, D = self.sino_shape
        if dtpl is not None:
            _dev(dtpl, (max(n_iter, 1),), torch.float64, "dtpl")
        prm = params.to_c()
        _check(_lib.osscir_mocca_iterate_noalloc(
            self._h, ctypes.byref(prm), _dev(state.f, (3, self.n, self.n), torch.float32, "f"),
            _dev(state.fbar, (3, self.n, self.n), torch.float32, "fbar"),
            _dev(state.y, (4, V, D), torch.float32, "y"), _dev(state.c, (4, V, D), torch.float32, "c"),
            int(n_iter), _dev(dtpl) if dtpl is not None else None, _stream_handle(stream)))
        return dtpl

    def mocca_stage(self, state: State, params: Params, stage: int, stream=None):
        """One stage (0 forward projection, 1 spectral + dual, 2 back-projection + primal)."""
        st = self._c_state(state)
        prm = params.to_c()
        _check(_lib.osscir_mocca_stage(self._h, ctypes.byref(prm), ctypes.byref(st), int(stage),
                                       _stream_handle(stream)))

    def ray_nnz(self, stream=None):
        """Number of pixels each ray crosses (int32 [V, D] device tensor)."""
        import torch
        out = torch.empty(*self.sino_shape, dtype=torch.int32, device="cuda")
        _check(_lib.osscir_ray_nnz(self._h, _dev(out), _stream_handle(stream)))
        return out

    def dtpl(self, f, c, work=None, stream=None):
        """D_TPL(c, chat(f)) as a 0-d float64 device tensor."""
        import torch
        work = self.workspace() if work is None else work
        out = torch.empty((), dtype=torch.float64, device="cuda")
        _check(_lib.osscir_dtpl(self._h, _dev(f, (3, self.n, self.n), torch.float32, "f"),
                                _dev(c, (4, *self.sino_shape), torch.float32, "c"), _dev(out), _dev(work),
                                work.numel(), _stream_handle(stream)))
        return out


def _c_geometry(geom) -> _Geometry:
    return _Geometry(int(geom.n), float(geom.pixel_cm), int(geom.n_views), int(geom.n_bins), float(geom.sid_cm),
                     float(geom.sdd_cm), float(geom.bin_cm), float(getattr(geom, "view0_rad", 0.0)),
                     float(getattr(geom, "arc_rad", 2 * np.pi)))


def ray_table(geom):
    """(rays [L, 6], src [V, 2]): the line parameters a plan of this geometry
    uses (host computation in the library, no device)."""
    lib = load_library()
    g = _c_geometry(geom)
    rays = np.zeros((int(geom.n_views) * int(geom.n_bins), 6))
    src = np.zeros((int(geom.n_views), 2))
    _check(lib.osscir_ray_table(ctypes.byref(g), rays.ctypes.data_as(_dp), src.ctypes.data_as(_dp)))
    return rays, src


def mu_pc_basis(spec):
    """(B [3, 3], mu~ [3, I]) of mu-preconditioning: mu~ = B mu orthonormal in
    energy; maps f = B^T g.  Host computation in the library."""
    lib = load_library()
    mu = np.ascontiguousarray(spec.mu, dtype=np.float64)
    s = np.ascontiguousarray(spec.s, dtype=np.float64)
    n0 = np.ascontiguousarray(spec.n0, dtype=np.float64)
    if s.ndim != 2:
        raise ValueError("mu-PC needs one shared window response s [W, I]")
    sp = _Spectral(mu.shape[0], s.shape[0], s.shape[1], mu.ctypes.data_as(_dp), s.ctypes.data_as(_dp),
                   n0.ctypes.data_as(_dp), 1, None)
    B = np.zeros((3, 3))
    mu_t = np.zeros_like(mu)
    _check(lib.osscir_mu_pc_basis(ctypes.byref(sp), B.ctypes.data_as(_dp), mu_t.ctypes.data_as(_dp)))
    return B, mu_t


def mu_pc_spectral(spec):
    """The spectral description with mu~ in place of mu, and B."""
    import types
    B, mu_t = mu_pc_basis(spec)
    return types.SimpleNamespace(mu=mu_t, s=np.asarray(spec.s), n0=np.asarray(spec.n0)), B


def material_transform(M, x, out=None, stream=None):
    """out = M x for [3, n, n] maps (M a 3x3 host matrix)."""
    import torch
    lib = load_library()
    Mc = np.ascontiguousarray(M, dtype=np.float64).reshape(3, 3)
    xp = _dev(x, None, torch.float32, "x")
    if x.shape[0] != 3:
        raise ValueError("x must have 3 channels")
    out = torch.empty_like(x) if out is None else out
    _check(lib.osscir_material_transform(Mc.ctypes.data_as(_dp), xp, _dev(out, tuple(x.shape), torch.float32, "out"),
                                         int(x[0].numel()), _stream_handle(stream)))
    return out


BATCH_CONFIG_FIELDS = [name for name, _ in _BatchConfig._fields_]


class Batch:
    """Many scans advanced together, one launch per stage for the whole batch.

    Slots hold (plan, state, lambda, max_iter, tol); modes (precond,
    curvature, fp64_small) are shared.  The binding keeps the bound plans and
    states alive while they are bound.
    """

    def __init__(self, modes: Params, max_slots: int):
        lib = load_library()
        h = c_void_p()
        prm = modes.to_c()
        _check(lib.osscir_batch_create(ctypes.byref(prm), int(max_slots), ctypes.byref(h)))
        self._h = h
        self.max_slots = int(max_slots)
        self._bound = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(_lib.osscir_batch_destroy(self._h))
            self._h = None
            self._bound = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_slot(self, slot: int, plan: Plan, state: State, lam: float, max_iter: int = 0, tol: float = 0.0,
                 stream=None, n_inner: int = 1, p0=None):
        """Bind a scan to a slot.  n_inner > 1: nested loops (as
        Plan.mocca_iterate_nested), with p0 an optional [3, V, D] float32
        device tensor the slot keeps X f0 in (allocated if None)."""
        import torch
        st = plan._c_state(state)
        if n_inner > 1:
            V, D = plan.sino_shape
            if p0 is None:
                p0 = torch.empty((3, V, D), dtype=torch.float32, device="cuda")
            p0_ptr = _dev(p0, (3, V, D), torch.float32, "p0")
        else:
            p0, p0_ptr = None, None
        _check(_lib.osscir_batch_set_slot_nested(self._h, int(slot), plan._h, ctypes.byref(st), float(lam),
                                                 int(max_iter), float(tol), int(n_inner), p0_ptr,
                                                 _stream_handle(stream)))
        self._bound[int(slot)] = (plan, state, p0)

    def clear_slot(self, slot: int):
        _check(_lib.osscir_batch_clear_slot(self._h, int(slot)))
        self._bound.pop(int(slot), None)

    def iterate(self, n_iter: int, use_graph: bool = True, stream=None):
        _check(_lib.osscir_batch_iterate(self._h, int(n_iter), int(bool(use_graph)), _stream_handle(stream)))

    def status(self, stream=None):
        """List of (state, iters, rel_change) per slot (synchronises the stream)."""
        arr = (_SlotStatus * self.max_slots)()
        _check(_lib.osscir_batch_status(self._h, arr, _stream_handle(stream)))
        return [(a.state, a.iters, a.rel_change) for a in arr]

    def get_config(self) -> dict:
        c = _BatchConfig()
        _check(_lib.osscir_batch_get_config(self._h, ctypes.byref(c)))
        return {k: int(getattr(c, k)) for k in BATCH_CONFIG_FIELDS}

    def set_config(self, **kw):
        cfg = self.get_config()
        cfg.update(kw)
        c = _BatchConfig(*[int(cfg[k]) for k in BATCH_CONFIG_FIELDS])
        _check(_lib.osscir_batch_set_config(self._h, ctypes.byref(c)))

    def tune(self, iters_per_trial: int = 2, stream=None) -> dict:
        c = _BatchConfig()
        _check(_lib.osscir_batch_tune(self._h, int(iters_per_trial), ctypes.byref(c), _stream_handle(stream)))
        return {k: int(getattr(c, k)) for k in BATCH_CONFIG_FIELDS}


def version() -> str:
    return load_library().osscir_version().decode()

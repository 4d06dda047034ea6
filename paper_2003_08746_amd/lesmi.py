"""Python binding of the C ABI in include/les.h (argument marshalling only).

Every step of the method runs in the HIP kernels of liblesmi.so; this module
only converts arguments.  torch supplies device memory and the current HIP
stream.  There is no CPU fallback: importing works without a GPU (for
inspection), but every call that computes needs the built library and a
gfx950 device, and raises otherwise.

The functions keep the C names (les_create, les_residual, les_rk_step,
les_adjoint_step, ...).  ``Solver`` bundles a context with helpers that move
dense padded arrays in and out of the library layout.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblesmi.so")

LES_OK, LES_ERR_ARG, LES_ERR_HIP, LES_ERR_NOMEM, LES_ERR_NONFINITE, LES_ERR_STATE = 0, -1, -2, -3, -4, -5
LES_FP64, LES_MIXED = 0, 1
LES_BC_PERIODIC, LES_BC_DIRICHLET, LES_BC_PERIODIC_SUPERPOSED, LES_BC_AXIS = 0, 1, 2, 3
LES_FACE_FROZEN, LES_FACE_CHARACTERISTIC, LES_FACE_EXIT, LES_FACE_FARFIELD = 0, 1, 2, 3

EXPORTED = ["les_create", "les_destroy", "les_layout", "les_layout_for", "les_get_metrics", "les_residual",
            "les_cfl_dt", "les_set_forcing", "les_rk_step", "les_advance", "les_adjoint_step", "les_residual_adjoint",
            "les_probe_objective", "les_set_face", "les_stats_accumulate", "les_stats_profiles",
            "les_residual_noalloc", "les_last_error", "les_last_create_error"]

# fields of les_stats_accumulate, in its order (sums over k of each)
LES_STATS_NF = 12
STATS_FIELDS = ("rho", "u", "v", "w", "p", "uu", "vv", "ww", "uv", "uw", "vw", "pp")
# fields of les_stats_profiles, in its order
LES_PROF_NF = 10
PROF_FIELDS = ("rho", "u", "v", "w", "p", "u_rms", "v_rms", "w_rms", "p_rms", "uv")


class LesError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class LesGrid(ctypes.Structure):
    _fields_ = [("ni", ctypes.c_int), ("nj", ctypes.c_int), ("nk", ctypes.c_int), ("bc", ctypes.c_int * 3),
                ("xyz", ctypes.c_void_p)]


class LesMetrics(ctypes.Structure):
    _fields_ = [("m", ctypes.c_void_p)]


class LesFlowParams(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("Pr", ctypes.c_double), ("Pr_sgs", ctypes.c_double),
                ("mu_ref", ctypes.c_double), ("T_ref", ctypes.c_double), ("S_suth", ctypes.c_double),
                ("R_gas", ctypes.c_double), ("sgs", ctypes.c_int), ("Cs", ctypes.c_double),
                ("k2", ctypes.c_double), ("k4", ctypes.c_double), ("alpha", ctypes.c_double),
                ("cfl", ctypes.c_double), ("prec", ctypes.c_int), ("CI", ctypes.c_double)]


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_llp = ctypes.POINTER(ctypes.c_longlong)


def lib():
    """Load liblesmi.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    L.les_create.restype = ctypes.c_int
    L.les_create.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(LesGrid), ctypes.POINTER(LesMetrics),
                             ctypes.POINTER(LesFlowParams), _vp]
    L.les_destroy.restype = None
    L.les_destroy.argtypes = [_vp]
    L.les_layout.restype = ctypes.c_int
    L.les_layout.argtypes = [_vp, _llp, _llp, _llp, ctypes.POINTER(ctypes.c_int)]
    L.les_layout_for.restype = ctypes.c_int
    L.les_layout_for.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _llp, _llp, _llp,
                                 ctypes.POINTER(ctypes.c_int)]
    L.les_get_metrics.restype = ctypes.c_int
    L.les_get_metrics.argtypes = [_vp, _vp]
    L.les_residual.restype = ctypes.c_int
    L.les_residual.argtypes = [_vp, _vp, _vp, _dp]
    L.les_cfl_dt.restype = ctypes.c_int
    L.les_cfl_dt.argtypes = [_vp, _vp, _dp]
    L.les_set_forcing.restype = ctypes.c_int
    L.les_set_forcing.argtypes = [_vp, _vp, ctypes.c_int]
    L.les_rk_step.restype = ctypes.c_int
    L.les_rk_step.argtypes = [_vp, _vp, ctypes.c_double, _dp, _dp, _vp]
    L.les_residual_noalloc.restype = ctypes.c_int
    L.les_residual_noalloc.argtypes = [_vp, _vp, _vp, _vp]
    L.les_advance.restype = ctypes.c_int
    L.les_advance.argtypes = [_vp, _vp, ctypes.c_int, _dp, _dp]
    L.les_adjoint_step.restype = ctypes.c_int
    L.les_adjoint_step.argtypes = [_vp, _vp, ctypes.c_double, _vp, _vp]
    L.les_residual_adjoint.restype = ctypes.c_int
    L.les_residual_adjoint.argtypes = [_vp, _vp, _vp, _vp]
    L.les_probe_objective.restype = ctypes.c_int
    L.les_probe_objective.argtypes = [_vp, _vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, _vp, _vp]
    L.les_set_face.restype = ctypes.c_int
    L.les_set_face.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_double]
    L.les_stats_accumulate.restype = ctypes.c_int
    L.les_stats_accumulate.argtypes = [_vp, _vp, _vp]
    L.les_stats_profiles.restype = ctypes.c_int
    L.les_stats_profiles.argtypes = [_vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp, _vp]
    L.les_last_error.restype = ctypes.c_char_p
    L.les_last_error.argtypes = [_vp]
    L.les_last_create_error.restype = ctypes.c_char_p
    L.les_last_create_error.argtypes = []
    L.les_debug_use_reference.restype = ctypes.c_int
    L.les_debug_use_reference.argtypes = [_vp, ctypes.c_int]
    L.les_debug_stage_timing.restype = ctypes.c_int
    L.les_debug_stage_timing.argtypes = [_vp, ctypes.c_int]
    L.les_debug_stage_time.restype = ctypes.c_int
    L.les_debug_stage_time.argtypes = [_vp, _dp, ctypes.POINTER(ctypes.c_longlong)]
    L.les_debug_dynamic_coefficients.restype = ctypes.c_int
    L.les_debug_dynamic_coefficients.argtypes = [_vp, _vp, _vp]
    L.les_debug_stream_copy.restype = ctypes.c_int
    L.les_debug_stream_copy.argtypes = [_vp, _vp, ctypes.c_longlong, _vp]
    _lib = L
    return L


def _check(rc, ctx=None, what=""):
    if rc != LES_OK:
        L = lib()
        msg = (L.les_last_error(ctx) if ctx else L.les_last_create_error()) or b""
        raise LesError(rc, f"{what}: {msg.decode(errors='replace')}")


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream_ptr(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def flow_params_struct(p: dict, prec: int = LES_FP64) -> LesFlowParams:
    s = LesFlowParams()
    for k in ["gamma", "Pr", "Pr_sgs", "mu_ref", "T_ref", "S_suth", "R_gas", "Cs", "k2", "k4", "alpha", "cfl"]:
        setattr(s, k, float(p[k]))
    s.CI = float(p.get("CI", 0.0))
    s.sgs = int(p["sgs"])
    s.prec = int(prec)
    return s


# ---------------------------------------------------------------------------
# C names
# ---------------------------------------------------------------------------
def les_create(grid: LesGrid, metrics_ptr, params: LesFlowParams, stream_ptr) -> int:
    """metrics_ptr: device pointer of caller metrics (dense padded [10][..])
    or None to compute them from grid.xyz."""
    ctx = _vp()
    m = None
    if metrics_ptr is not None:
        m = LesMetrics()
        m.m = metrics_ptr
    rc = lib().les_create(ctypes.byref(ctx), ctypes.byref(grid), None if m is None else ctypes.byref(m),
                          ctypes.byref(params), stream_ptr)
    _check(rc, None, "les_create")
    return ctx.value


def les_destroy(ctx) -> None:
    lib().les_destroy(ctx)


def les_layout(ctx):
    """(strides, origin, field_elems, ghost)"""
    st = (ctypes.c_longlong * 3)()
    o = ctypes.c_longlong()
    fe = ctypes.c_longlong()
    gh = ctypes.c_int()
    _check(lib().les_layout(ctx, st, ctypes.byref(o), ctypes.byref(fe), ctypes.byref(gh)), ctx, "les_layout")
    return tuple(st), o.value, fe.value, gh.value


def les_layout_for(ni, nj, nk):
    """(strides, origin, field_elems, ghost)"""
    st = (ctypes.c_longlong * 3)()
    o = ctypes.c_longlong()
    fe = ctypes.c_longlong()
    gh = ctypes.c_int()
    _check(lib().les_layout_for(ni, nj, nk, st, ctypes.byref(o), ctypes.byref(fe), ctypes.byref(gh)), None,
           "les_layout_for")
    return tuple(st), o.value, fe.value, gh.value


def les_get_metrics(ctx, dense_out_ptr):
    _check(lib().les_get_metrics(ctx, dense_out_ptr), ctx, "les_get_metrics")


def les_residual(ctx, Q_ptr, R_ptr, want_norms=False):
    norms = (ctypes.c_double * 10)() if want_norms else None
    rc = lib().les_residual(ctx, Q_ptr, R_ptr, norms)
    _check(rc, ctx, "les_residual")
    return np.array(norms[:]) if want_norms else None


def les_cfl_dt(ctx, Q_ptr) -> float:
    dt = ctypes.c_double()
    _check(lib().les_cfl_dt(ctx, Q_ptr, ctypes.byref(dt)), ctx, "les_cfl_dt")
    return dt.value


def les_set_forcing(ctx, f_ptr, i_f):
    _check(lib().les_set_forcing(ctx, f_ptr, int(i_f)), ctx, "les_set_forcing")


def les_rk_step(ctx, Q_ptr, dt=0.0, want_dt=False, want_norms=False, ckpt_ptr=None):
    dto = ctypes.c_double() if want_dt else None
    norms = (ctypes.c_double * 10)() if want_norms else None
    rc = lib().les_rk_step(ctx, Q_ptr, float(dt), ctypes.byref(dto) if want_dt else None, norms, ckpt_ptr)
    _check(rc, ctx, "les_rk_step")
    return (dto.value if want_dt else None), (np.array(norms[:]) if want_norms else None)


def les_residual_noalloc(ctx, Q_ptr, R_ptr, norms_dev_ptr=None):
    _check(lib().les_residual_noalloc(ctx, Q_ptr, R_ptr, norms_dev_ptr), ctx, "les_residual_noalloc")


def les_advance(ctx, Q_ptr, nsteps, want_dt=False, want_norms=False):
    dts = (ctypes.c_double * int(nsteps))() if want_dt else None
    norms = (ctypes.c_double * 10)() if want_norms else None
    rc = lib().les_advance(ctx, Q_ptr, int(nsteps), dts, norms)
    _check(rc, ctx, "les_advance")
    return (np.array(dts[:]) if want_dt else None), (np.array(norms[:]) if want_norms else None)


def les_adjoint_step(ctx, ckpt_ptr, dt, Qbar_ptr, fbar_ptr=None):
    _check(lib().les_adjoint_step(ctx, ckpt_ptr, float(dt), Qbar_ptr, fbar_ptr), ctx, "les_adjoint_step")


def les_residual_adjoint(ctx, Q_ptr, Rbar_ptr, Qbar_ptr):
    _check(lib().les_residual_adjoint(ctx, Q_ptr, Rbar_ptr, Qbar_ptr), ctx, "les_residual_adjoint")


def les_probe_objective(ctx, Q_ptr, i_p, p_inf, weight, J_ptr, Qbar_ptr=None):
    _check(lib().les_probe_objective(ctx, Q_ptr, int(i_p), float(p_inf), float(weight), J_ptr, Qbar_ptr), ctx,
           "les_probe_objective")


def les_set_face(ctx, face, type_, Q_outside_ptr=None, p_exit=0.0):
    _check(lib().les_set_face(ctx, int(face), int(type_), Q_outside_ptr, float(p_exit)), ctx, "les_set_face")


def les_stats_accumulate(ctx, Q_ptr, acc_ptr):
    _check(lib().les_stats_accumulate(ctx, Q_ptr, acc_ptr), ctx, "les_stats_accumulate")


def les_stats_profiles(ctx, acc_ptr, samples, u_jet, core_frac, prof_ptr, core_ptr):
    _check(lib().les_stats_profiles(ctx, acc_ptr, float(samples), float(u_jet), float(core_frac), prof_ptr,
                                    core_ptr), ctx, "les_stats_profiles")


def les_debug_use_reference(ctx, on: bool):
    _check(lib().les_debug_use_reference(ctx, 1 if on else 0), ctx, "les_debug_use_reference")


def les_debug_stage_timing(ctx, on: bool):
    _check(lib().les_debug_stage_timing(ctx, 1 if on else 0), ctx, "les_debug_stage_timing")


def les_debug_stage_time(ctx):
    ms = ctypes.c_double()
    n = ctypes.c_longlong()
    _check(lib().les_debug_stage_time(ctx, ctypes.byref(ms), ctypes.byref(n)), ctx, "les_debug_stage_time")
    return ms.value, n.value


def les_debug_stream_copy(src_ptr, dst_ptr, nbytes, stream_ptr=None):
    _check(lib().les_debug_stream_copy(src_ptr, dst_ptr, int(nbytes), stream_ptr), None, "les_debug_stream_copy")


# ---------------------------------------------------------------------------
# Convenience wrapper around one context
# ---------------------------------------------------------------------------
class Solver:
    """One block on one GPU.  ``case`` is a dict from ``inputs`` (ni, nj, nk,
    bc, xyz (dense padded numpy or torch), params)."""

    def __init__(self, case: dict, prec: int = LES_FP64, device: str = "cuda", stream=None, xyz=None, metrics=None):
        """metrics: optional caller metrics, a device float64 tensor in the
        dense padded layout (10, nk+4, nj+4, ni+4); then xyz is not read."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.ni, self.nj, self.nk = int(case["ni"]), int(case["nj"]), int(case["nk"])
        self.bc = tuple(int(b) for b in case["bc"])
        self.params = dict(case["params"])
        self.prec = prec
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        g = LesGrid()
        g.ni, g.nj, g.nk = self.ni, self.nj, self.nk
        for d in range(3):
            g.bc[d] = self.bc[d]
        xyz_t = None
        if metrics is None:
            if xyz is None:
                xyz = case["xyz"]
            xyz_t = xyz if isinstance(xyz, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(xyz))
            xyz_t = xyz_t.to(self.device, torch.float64).contiguous()
            g.xyz = xyz_t.data_ptr()
        else:
            assert metrics.dtype == torch.float64 and metrics.is_contiguous() and metrics.is_cuda
            assert metrics.shape == (10, self.nk + 4, self.nj + 4, self.ni + 4)
        with torch.cuda.stream(self.stream):
            self.ctx = les_create(g, None if metrics is None else metrics.data_ptr(),
                                  flow_params_struct(self.params, prec), int(self.stream.cuda_stream))
        del xyz_t
        self.strides, self.origin, self.fe, self.ghost = les_layout(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            les_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- memory helpers (layout marshalling) ---
    def empty_state(self, nf=5, dtype=None):
        t = self.torch
        return t.zeros(nf * self.fe, dtype=dtype or t.float64, device=self.device)

    def view(self, state, nf=5):
        """Dense padded view (nf, nk+4, nj+4, ni+4) of a library-layout array."""
        sj, sk, g = self.strides[1], self.strides[2], self.ghost
        start = self.origin - g - g * sj - g * sk
        return state.as_strided((nf, self.nk + 2 * g, self.nj + 2 * g, self.ni + 2 * g), (self.fe, sk, sj, 1),
                                state.storage_offset() + start)

    def upload(self, dense, nf=5):
        t = self.torch
        st = self.empty_state(nf)
        src = dense if isinstance(dense, t.Tensor) else t.from_numpy(np.ascontiguousarray(dense))
        self.view(st, nf).copy_(src.to(self.device, t.float64))
        return st

    def download(self, state, nf=5) -> np.ndarray:
        return self.view(state, nf).cpu().numpy().copy()

    def metrics_dense(self) -> np.ndarray:
        t = self.torch
        out = t.zeros((10, self.nk + 4, self.nj + 4, self.ni + 4), dtype=t.float64, device=self.device)
        les_get_metrics(self.ctx, out.data_ptr())
        return out.cpu().numpy()

    # --- method calls ---
    def residual(self, Q, want_norms=False):
        R = self.empty_state()
        norms = les_residual(self.ctx, Q.data_ptr(), R.data_ptr(), want_norms)
        return (R, norms) if want_norms else R

    def cfl_dt(self, Q) -> float:
        return les_cfl_dt(self.ctx, Q.data_ptr())

    def rk_step(self, Q, dt=0.0, want_dt=False, want_norms=False, ckpt=None):
        return les_rk_step(self.ctx, Q.data_ptr(), dt, want_dt, want_norms, _ptr(ckpt))

    def dynamic_coefficients(self, Q):
        """(C, D_T) per padded column, (nj+4, ni+4) numpy arrays, of the
        dynamic SGS closure at Q (instrumentation entry point)."""
        t = self.torch
        out = t.empty(2 * (self.nj + 4) * (self.ni + 4), dtype=t.float64, device=self.device)
        _check(lib().les_debug_dynamic_coefficients(self.ctx, Q.data_ptr(), out.data_ptr()), self.ctx,
               "les_debug_dynamic_coefficients")
        a = out.cpu().numpy().reshape(2, self.nj + 4, self.ni + 4)
        return a[0].copy(), a[1].copy()

    def advance(self, Q, nsteps, want_dt=False, want_norms=False):
        """nsteps CFL steps in one call (les_advance); returns (dts, norms)."""
        return les_advance(self.ctx, Q.data_ptr(), nsteps, want_dt, want_norms)

    def set_forcing(self, f, i_f):
        les_set_forcing(self.ctx, None if f is None else f.data_ptr(), i_f)

    def adjoint_step(self, ckpt, dt, Qbar, fbar=None):
        les_adjoint_step(self.ctx, ckpt.data_ptr(), dt, Qbar.data_ptr(), _ptr(fbar))

    def residual_adjoint(self, Q, Rbar):
        Qbar = self.empty_state()
        les_residual_adjoint(self.ctx, Q.data_ptr(), Rbar.data_ptr(), Qbar.data_ptr())
        return Qbar

    def probe_objective(self, Q, i_p, p_inf, weight, J, Qbar=None):
        les_probe_objective(self.ctx, Q.data_ptr(), i_p, p_inf, weight, J.data_ptr(), _ptr(Qbar))

    def set_face(self, face, type_, Q_outside=None, p_exit=0.0):
        """Boundary face treatment (les_set_face); Q_outside: library-layout
        state whose ghost values are the outside state, or None."""
        les_set_face(self.ctx, face, type_, _ptr(Q_outside), p_exit)

    def stats_accumulate(self, Q, acc=None):
        """acc[s][j][i] += sums over k of STATS_FIELDS at the interior of Q;
        acc: device float64 (LES_STATS_NF, nj, ni), allocated (zero) when None."""
        t = self.torch
        if acc is None:
            acc = t.zeros((LES_STATS_NF, self.nj, self.ni), dtype=t.float64, device=self.device)
        assert acc.shape == (LES_STATS_NF, self.nj, self.ni) and acc.dtype == t.float64 and acc.is_contiguous()
        les_stats_accumulate(self.ctx, Q.data_ptr(), acc.data_ptr())
        return acc

    @property
    def stats_planes(self) -> int:
        """k planes one les_stats_accumulate call sums: nk, or nk - 1 along a
        superposed k direction (its last plane repeats the first)."""
        return self.nk - 1 if self.bc[2] == LES_BC_PERIODIC_SUPERPOSED else self.nk

    def stats_profiles(self, acc, samples, u_jet=None, core_frac=0.95):
        """Mean-flow and RMS profiles (les_stats_profiles) from the sums in
        acc; samples = number of accumulations times stats_planes.  Returns a dict of
        (nj, ni) device tensors keyed by PROF_FIELDS, plus "core" (a bool
        (nj, ni) tensor: the potential core, <u> >= core_frac u_jet) when
        u_jet is given."""
        t = self.torch
        assert acc.shape == (LES_STATS_NF, self.nj, self.ni) and acc.dtype == t.float64 and acc.is_contiguous()
        prof = t.empty((LES_PROF_NF, self.nj, self.ni), dtype=t.float64, device=self.device)
        core = None if u_jet is None else t.empty((self.nj, self.ni), dtype=t.uint8, device=self.device)
        les_stats_profiles(self.ctx, acc.data_ptr(), samples, 0.0 if u_jet is None else u_jet, core_frac,
                           prof.data_ptr(), _ptr(core))
        out = {name: prof[f] for f, name in enumerate(PROF_FIELDS)}
        if core is not None:
            out["core"] = core.bool()
        return out

    def use_reference(self, on=True):
        les_debug_use_reference(self.ctx, on)

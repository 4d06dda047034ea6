"""ctypes wrapper of the plain FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU path: it loads
``liboracle.so`` built from ``les_oracle.cpp`` (see ``build.py``), which
implements the residual and Runge-Kutta step of the paper's Sec. 3-4 with the
readings listed at the top of that file.

Array conventions (numpy, float64, C-contiguous):
  * padded box arrays have shape (nfields, nk+4, nj+4, ni+4): two ghost layers
    per side, i fastest; interior index 0..n-1 sits at n+2;
  * coordinates xyz: (3, ...); metrics: (10, ...) = xi_x/J .. zeta_z/J, J;
  * state Q: (5, ...) = rho, rho u, rho v, rho w, e;
  * source f: (5, nk, nj) on the plane i = i_f.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


class OrcDims(ctypes.Structure):
    _fields_ = [("ni", ctypes.c_int), ("nj", ctypes.c_int), ("nk", ctypes.c_int),
                ("bc", ctypes.c_int * 3), ("face", ctypes.c_int * 6), ("p_exit", ctypes.c_double * 6),
                ("outside", ctypes.c_void_p)]


class OrcParams(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("Pr", ctypes.c_double), ("Pr_sgs", ctypes.c_double),
                ("mu_ref", ctypes.c_double), ("T_ref", ctypes.c_double), ("S_suth", ctypes.c_double),
                ("R_gas", ctypes.c_double), ("sgs", ctypes.c_int), ("Cs", ctypes.c_double),
                ("k2", ctypes.c_double), ("k4", ctypes.c_double), ("alpha", ctypes.c_double),
                ("cfl", ctypes.c_double), ("CI", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_box_nodes.restype = ctypes.c_size_t
    lib.orc_box_nodes.argtypes = [ctypes.POINTER(OrcDims)]
    lib.orc_metrics.restype = None
    lib.orc_metrics.argtypes = [ctypes.POINTER(OrcDims), _dp, _dp]
    lib.orc_fill_ghosts.restype = None
    lib.orc_fill_ghosts.argtypes = [ctypes.POINTER(OrcDims), _dp, ctypes.c_int]
    lib.orc_residual.restype = None
    lib.orc_residual.argtypes = [ctypes.POINTER(OrcDims), ctypes.POINTER(OrcParams), _dp, _dp, _dp,
                                 ctypes.c_int, _dp]
    lib.orc_residual_tangent.restype = None
    lib.orc_residual_tangent.argtypes = [ctypes.POINTER(OrcDims), ctypes.POINTER(OrcParams), _dp, _dp, _dp,
                                         _dp, _dp, ctypes.c_int, _dp, _dp]
    lib.orc_cfl_dt.restype = ctypes.c_double
    lib.orc_cfl_dt.argtypes = [ctypes.POINTER(OrcDims), ctypes.POINTER(OrcParams), _dp, _dp]
    lib.orc_rk_step.restype = ctypes.c_double
    lib.orc_rk_step.argtypes = [ctypes.POINTER(OrcDims), ctypes.POINTER(OrcParams), _dp, _dp, ctypes.c_double,
                                _dp, ctypes.c_int, _dp, _dp]
    lib.orc_rk_step_tangent.restype = None
    lib.orc_rk_step_tangent.argtypes = [ctypes.POINTER(OrcDims), ctypes.POINTER(OrcParams), _dp, _dp, _dp,
                                        ctypes.c_double, _dp, _dp, ctypes.c_int]
    lib.orc_objective_rollout.restype = ctypes.c_double
    lib.orc_objective_rollout.argtypes = [ctypes.POINTER(OrcDims), ctypes.POINTER(OrcParams), _dp, _dp, _dp,
                                          _dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_double, _dp]
    lib.orc_objective.restype = ctypes.c_double
    lib.orc_objective.argtypes = [ctypes.POINTER(OrcDims), ctypes.POINTER(OrcParams), _dp, _dp, _dp,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double]
    lib.orc_fill_ghosts_faces.restype = None
    lib.orc_fill_ghosts_faces.argtypes = [ctypes.POINTER(OrcDims), ctypes.POINTER(OrcParams), _dp, _dp]
    lib.orc_stats.restype = None
    lib.orc_stats.argtypes = [ctypes.POINTER(OrcDims), ctypes.POINTER(OrcParams), _dp, _dp]
    lib.orc_stats_profiles.restype = None
    lib.orc_stats_profiles.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, _dp, ctypes.c_void_p]
    lib.orc_dynamic_coefficients.restype = None
    lib.orc_dynamic_coefficients.argtypes = [ctypes.POINTER(OrcDims), ctypes.POINTER(OrcParams), _dp, _dp, _dp, _dp]
    lib.orc_residual_nofill.restype = None
    lib.orc_residual_nofill.argtypes = [ctypes.POINTER(OrcDims), ctypes.POINTER(OrcParams), _dp, _dp, _dp]
    lib.orc_threads.restype = ctypes.c_int
    lib.orc_threads.argtypes = [ctypes.c_int]
    lib.orc_rk_scalar.restype = None
    lib.orc_rk_scalar.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, _dp]
    _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def threads(n: int = 0) -> int:
    """Set the oracle's OpenMP thread count (n > 0) and return the count its
    loops use."""
    return int(_load().orc_threads(int(n)))


def dims(ni, nj, nk, bc=(0, 0, 0)) -> OrcDims:
    d = OrcDims()
    d.ni, d.nj, d.nk = int(ni), int(nj), int(nk)
    for i in range(3):
        d.bc[i] = int(bc[i])
    return d


_PARAM_KEYS = ["gamma", "Pr", "Pr_sgs", "mu_ref", "T_ref", "S_suth", "R_gas", "sgs", "Cs", "k2", "k4",
               "alpha", "cfl", "CI"]


def params(p: dict) -> OrcParams:
    o = OrcParams()
    for k in _PARAM_KEYS:
        setattr(o, k, int(p[k]) if k == "sgs" else float(p[k]))
    return o


# boundary-face types of a Dirichlet direction (faces i-lo, i-hi, j-lo, j-hi,
# k-lo, k-hi): frozen ghosts, characteristic entrance, exit, far field
FACE_FROZEN, FACE_CHARACTERISTIC, FACE_EXIT, FACE_FARFIELD = 0, 1, 2, 3


def _dims_of(case):
    """orc_dims of a case; case["faces"] (optional) = dict(types=[6],
    p_exit=[6], outside=padded (5, ...) state whose ghost values are the
    outside state of characteristic and far-field faces)."""
    d = dims(case["ni"], case["nj"], case["nk"], case["bc"])
    fc = case.get("faces")
    if fc:
        for f in range(6):
            d.face[f] = int(fc["types"][f])
            d.p_exit[f] = float(fc.get("p_exit", [0.0] * 6)[f])
        out = fc.get("outside")
        if out is not None:
            out = _pad(case, out, 5)
            assert out.shape == (5, case["nk"] + 4, case["nj"] + 4, case["ni"] + 4)
            d._outside_ref = out  # keep alive while d is used
            d.outside = out.ctypes.data
    return d


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _pad(case, a, nf=None):
    """a as a contiguous float64 array of shape (nf, nk+4, nj+4, ni+4) for
    the block of case (any nf when None): the C code trusts the shapes, so
    a mismatch is refused here instead of read out of bounds."""
    a = _c(a)
    want = (case["nk"] + 4, case["nj"] + 4, case["ni"] + 4)
    if a.ndim != 4 or a.shape[1:] != want or (nf is not None and a.shape[0] != nf):
        raise ValueError(f"oracle: array of shape {a.shape} for a block wanting ({nf}, {want[0]}, {want[1]}, {want[2]})")
    return a


def _forc(case, f):
    """A forcing plane array (5, nk, nj), contiguous float64, shape checked."""
    f = _c(f)
    if f.shape != (5, case["nk"], case["nj"]):
        raise ValueError(f"oracle: forcing of shape {f.shape}, want (5, {case['nk']}, {case['nj']})")
    return f


def metrics(case) -> np.ndarray:
    """Metrics (10, nk+4, nj+4, ni+4) from the coordinates case['xyz'];
    defined on nodes with all indices in [-1, n], NaN elsewhere."""
    lib = _load()
    xyz = _pad(case, case["xyz"], 3)
    m = np.empty((10,) + xyz.shape[1:], dtype=np.float64)
    lib.orc_metrics(ctypes.byref(_dims_of(case)), _ptr(xyz), _ptr(m))
    return m


def fill_ghosts(case, a: np.ndarray) -> np.ndarray:
    lib = _load()
    a = _pad(case, a).copy()
    lib.orc_fill_ghosts(ctypes.byref(_dims_of(case)), _ptr(a), a.shape[0])
    return a


def fill_ghosts_faces(case, m, Q, prm=None) -> np.ndarray:
    """Copy of Q with its ghosts filled: periodic wrap, frozen Dirichlet
    ghosts and the boundary faces of case["faces"]."""
    lib = _load()
    prm = case["params"] if prm is None else prm
    q = _pad(case, Q, 5).copy()
    lib.orc_fill_ghosts_faces(ctypes.byref(_dims_of(case)), ctypes.byref(params(prm)), _ptr(_pad(case, m, 10)), _ptr(q))
    return q


def residual(case, m, Q, prm=None, f=None, i_f=-1) -> np.ndarray:
    """R(Q) on the padded box (zeros in the ghost layers)."""
    lib = _load()
    prm = case["params"] if prm is None else prm
    Q = _pad(case, Q, 5)
    R = np.zeros_like(Q)
    fa = None if f is None else _forc(case, f)
    lib.orc_residual(ctypes.byref(_dims_of(case)), ctypes.byref(params(prm)), _ptr(_pad(case, m, 10)), _ptr(Q), _ptr(fa),
                     int(i_f), _ptr(R))
    return R


def residual_nofill(case, m, Q, prm=None) -> np.ndarray:
    """R(Q) with Q's ghost layers and axis nodes taken as given (no fill)."""
    lib = _load()
    prm = case["params"] if prm is None else prm
    Q = _pad(case, Q, 5)
    R = np.zeros_like(Q)
    lib.orc_residual_nofill(ctypes.byref(_dims_of(case)), ctypes.byref(params(prm)), _ptr(_pad(case, m, 10)), _ptr(Q), _ptr(R))
    return R


def residual_tangent(case, m, Q, dQ, prm=None, f=None, df=None, i_f=-1):
    """(R, dR) with dR the exact directional derivative of R along (dQ, df)."""
    lib = _load()
    prm = case["params"] if prm is None else prm
    Q = _pad(case, Q, 5)
    R = np.zeros_like(Q)
    dR = np.zeros_like(Q)
    lib.orc_residual_tangent(ctypes.byref(_dims_of(case)), ctypes.byref(params(prm)), _ptr(_pad(case, m, 10)), _ptr(Q),
                             _ptr(None if dQ is None else _pad(case, dQ, 5)), _ptr(None if f is None else _forc(case, f)),
                             _ptr(None if df is None else _forc(case, df)), int(i_f), _ptr(R), _ptr(dR))
    return R, dR


def dynamic_coefficients(case, m, Q, prm=None):
    """(C, D_T): the dynamic closure's coefficients per padded column, arrays
    (nj+4, ni+4) (mu_sgs = C rho D^2 |S|, kappa_sgs = Cp D_T rho D^2 |S|)."""
    lib = _load()
    prm = case["params"] if prm is None else prm
    C = np.zeros((case["nj"] + 4, case["ni"] + 4))
    D = np.zeros_like(C)
    lib.orc_dynamic_coefficients(ctypes.byref(_dims_of(case)), ctypes.byref(params(prm)), _ptr(_pad(case, m, 10)),
                                 _ptr(_pad(case, Q, 5)), _ptr(C), _ptr(D))
    return C, D


def cfl_dt(case, m, Q, prm=None) -> float:
    lib = _load()
    prm = case["params"] if prm is None else prm
    return lib.orc_cfl_dt(ctypes.byref(_dims_of(case)), ctypes.byref(params(prm)), _ptr(_pad(case, m, 10)), _ptr(_pad(case, Q, 5)))


def rk_step(case, m, Q, dt=0.0, prm=None, f=None, i_f=-1, want_stages=False):
    """One RK step from Q (not modified).  Returns (Q_next, dt, norms[10], stages|None)."""
    lib = _load()
    prm = case["params"] if prm is None else prm
    Qn = _pad(case, Q, 5).copy()
    norms = np.zeros(10, dtype=np.float64)
    stages = np.zeros((5,) + Qn.shape, dtype=np.float64) if want_stages else None
    dt_used = lib.orc_rk_step(ctypes.byref(_dims_of(case)), ctypes.byref(params(prm)), _ptr(_pad(case, m, 10)), _ptr(Qn),
                              float(dt), _ptr(None if f is None else _forc(case, f)), int(i_f), _ptr(norms), _ptr(stages))
    return Qn, dt_used, norms, stages


def rk_step_tangent(case, m, Q, dQ, dt, f=None, df=None, i_f=-1):
    """One RK step at fixed dt with its exact tangent: returns (Q_next, dQ_next)."""
    lib = _load()
    Qn = _pad(case, Q, 5).copy()
    dQn = _pad(case, dQ, 5).copy()
    lib.orc_rk_step_tangent(ctypes.byref(_dims_of(case)), ctypes.byref(params(case["params"])), _ptr(_pad(case, m, 10)),
                            _ptr(Qn), _ptr(dQn), float(dt), _ptr(None if f is None else _forc(case, f)),
                            _ptr(None if df is None else _forc(case, df)), int(i_f))
    return Qn, dQn


def objective_rollout(case, m, Q0, f, df, i_f, i_p, p_inf, nsteps, dt, dQ0=None):
    """(J, dJ): objective of the forcing workload and its exact directional
    derivative along (dQ0, df) computed with dual numbers."""
    lib = _load()
    prm = case["params"]
    Q = _pad(case, Q0, 5).copy()
    dJ = ctypes.c_double(0.0)
    J = lib.orc_objective_rollout(ctypes.byref(_dims_of(case)), ctypes.byref(params(prm)), _ptr(_pad(case, m, 10)), _ptr(Q),
                                  _ptr(None if dQ0 is None else _pad(case, dQ0, 5)), _ptr(_forc(case, f)),
                                  _ptr(None if df is None else _forc(case, df)), int(i_f), int(i_p), float(p_inf),
                                  int(nsteps), float(dt), ctypes.byref(dJ))
    return J, dJ.value


def objective(case, m, Q0, f, i_f, i_p, p_inf, nsteps, dt):
    lib = _load()
    Q = _pad(case, Q0, 5).copy()
    return lib.orc_objective(ctypes.byref(_dims_of(case)), ctypes.byref(params(case["params"])), _ptr(_pad(case, m, 10)),
                             _ptr(Q), _ptr(_forc(case, f)), int(i_f), int(i_p), float(p_inf), int(nsteps), float(dt))


def rk_scalar(lam: complex, dt: float, y0: complex = 1.0) -> complex:
    """The RK driver applied to y' = lam*y for one step."""
    lib = _load()
    yr = ctypes.c_double(float(np.real(y0)))
    yi = ctypes.c_double(float(np.imag(y0)))
    lib.orc_rk_scalar(float(np.real(lam)), float(np.imag(lam)), float(dt), ctypes.byref(yr), ctypes.byref(yi))
    return complex(yr.value, yi.value)


STATS_FIELDS = ("rho", "u", "v", "w", "p", "uu", "vv", "ww", "uv", "uw", "vw", "pp")


def stats(case, Q, acc=None, prm=None) -> np.ndarray:
    """Running statistics (Sec. 6 mean-flow and RMS profiles, averaged over
    time and the periodic direction k): acc[s][j][i] += sum_k phi_s, phi in
    STATS_FIELDS order, over the distinct k planes (nk - 1 of them along a
    superposed k direction).  Returns acc (a new zero array when acc is None)."""
    lib = _load()
    prm = case["params"] if prm is None else prm
    if acc is None:
        acc = np.zeros((len(STATS_FIELDS), case["nj"], case["ni"]))
    assert acc.shape == (len(STATS_FIELDS), case["nj"], case["ni"]) and acc.dtype == np.float64
    assert acc.flags.c_contiguous
    lib.orc_stats(ctypes.byref(_dims_of(case)), ctypes.byref(params(prm)), _ptr(_pad(case, Q, 5)), _ptr(acc))
    return acc


PROF_FIELDS = ("rho", "u", "v", "w", "p", "u_rms", "v_rms", "w_rms", "p_rms", "uv")


def stats_profiles(acc, samples, u_jet=1.0, core_frac=0.95):
    """Sec. 6 profiles from the sums of stats(): (prof, core) with prof of
    shape (10, nj, ni) in PROF_FIELDS order and core the potential-core mask
    (nj, ni) as uint8 (<u> >= core_frac u_jet)."""
    lib = _load()
    acc = _c(acc)
    nj, ni = acc.shape[1:]
    prof = np.zeros((len(PROF_FIELDS), nj, ni))
    core = np.zeros((nj, ni), dtype=np.uint8)
    lib.orc_stats_profiles(ni, nj, _ptr(acc), float(samples), float(u_jet), float(core_frac), _ptr(prof),
                           core.ctypes.data)
    return prof, core

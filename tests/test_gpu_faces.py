"""Boundary faces of a Dirichlet direction (les_set_face: characteristic
entrance, subsonic exit and far field, Sec. 3) against the oracle: the ghost
states, the residual, two RK steps in FP64 and in FP32-mixed, the argument
errors, and the adjoint through the face rules (dot-product tests against the
oracle's dual-number tangents).  Tolerances: the FP64 bar of 1e-12 relative to
each field's maximum; the mixed path's bound of 2e-6."""
import numpy as np
import pytest

from paper_2003_08746_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12
MIXED_BOUND = 2e-6


@pytest.fixture(scope="module")
def lesmi():
    import torch
    assert torch.cuda.is_available()
    from paper_2003_08746_amd import lesmi as L
    L.lib()
    return L


def _case(ni=61, nj=29, nk=23, seed=3):
    """Jet block, Dirichlet in i (entrance at i-lo, exit at i-hi) and j (far
    field on both sides), periodic in k; the interior is perturbed away from
    the outside state (the analytic jet profile with a small spanwise
    cross-flow, so that the far-field flow angle is not the normal's)."""
    c = I.jet_case(ni, nj, nk, seed=seed)
    c["bc"] = (1, 1, 0)
    g = c["params"]["gamma"]
    Q0 = I.outside_state(c, cross=(0.0, 0.0, 0.03))
    rng = np.random.default_rng(seed)
    Q = c["Q"].copy()
    Q[1:4] += 0.05 * rng.uniform(-1, 1, size=Q[1:4].shape)
    Q[4] *= 1.0 + 0.02 * rng.uniform(-1, 1, size=Q[4].shape)
    c["Q"] = Q
    c["faces"] = dict(types=[1, 2, 3, 3, 0, 0], p_exit=[0.0, 1.0 / g, 0, 0, 0, 0], outside=Q0)
    return c, Q0


def _solver(lesmi, case, Q0, prec=None):
    s = lesmi.Solver(case, prec=lesmi.LES_FP64 if prec is None else prec)
    fc = case["faces"]
    s.set_face(0, lesmi.LES_FACE_CHARACTERISTIC, s.upload(Q0))
    s.set_face(1, lesmi.LES_FACE_EXIT, p_exit=fc["p_exit"][1])
    s.set_face(2, lesmi.LES_FACE_FARFIELD)
    s.set_face(3, lesmi.LES_FACE_FARFIELD)
    return s


def _rel(a, b):
    ai, bi = I.interior(a), I.interior(b)
    den = np.abs(bi).reshape(bi.shape[0], -1).max(1)
    return np.abs(ai - bi).reshape(ai.shape[0], -1).max(1) / den


def test_face_ghosts_and_residual(orc, lesmi):
    import torch
    case, Q0 = _case()
    print("[gpu] faces: ghosts + residual 61x29x23", flush=True)
    s = _solver(lesmi, case, Q0)
    Q = s.upload(case["Q"])
    R = s.residual(Q)  # fills Q's ghosts in place
    torch.cuda.synchronize()
    Qg = s.download(Q)
    m = orc.metrics(case)
    Qo = orc.fill_ghosts_faces(case, m, case["Q"])
    scale = np.abs(Qo).reshape(5, -1).max(1)
    err = np.abs(Qg - Qo).reshape(5, -1).max(1) / scale  # every node, ghosts included
    assert (err <= 1e-13).all(), err
    Ro = orc.residual(case, m, case["Q"])
    assert (_rel(s.download(R), Ro) <= TOL).all(), _rel(s.download(R), Ro)
    s.close()


def test_face_jet_shard_residual(orc, lesmi):
    """The 256 x 128 x 128 jet shard with the faces the benchmark's faces leg
    times (entrance at i-lo, exit at i-hi, far field on both j sides): the
    whole residual per field to 1e-12 and the CFL step to 1e-14."""
    case, Q0 = _case(256, 128, 128, seed=0)
    print("[gpu] faces: residual 256x128x128", flush=True)
    s = _solver(lesmi, case, Q0)
    Q = s.upload(case["Q"])
    dt = s.cfl_dt(Q)
    Rg = s.download(s.residual(Q))
    s.close()
    m = orc.metrics(case)
    Ro = orc.residual(case, m, case["Q"])
    assert (_rel(Rg, Ro) <= TOL).all(), _rel(Rg, Ro)
    dto = orc.cfl_dt(case, m, case["Q"])
    assert abs(dt - dto) <= 1e-14 * dto, (dt, dto)


def test_face_rk_steps_fp64(orc, lesmi):
    case, Q0 = _case()
    print("[gpu] faces: 2 RK steps FP64", flush=True)
    m = orc.metrics(case)
    dt = 0.8 * orc.cfl_dt(case, m, case["Q"])
    s = _solver(lesmi, case, Q0)
    Q = s.upload(case["Q"])
    Qo = case["Q"]
    for _ in range(2):
        s.rk_step(Q, dt)
        Qo, _, _, _ = orc.rk_step(case, m, Qo, dt=dt)
    err = _rel(s.download(Q), Qo)
    assert (err <= TOL).all(), err
    s.close()


@pytest.mark.parametrize("sgs,CI", [(2, 0.0), (1, 0.05)])
def test_face_sgs_variants(orc, lesmi, sgs, CI):
    """The SGS variants with boundary faces: the dynamic closure's test
    filter and column sums read the face ghosts (ghost columns of the
    Dirichlet sides take the nearest interior column), and sigma_kk enters the
    flux pressure next to them; residual and two CFL steps in FP64."""
    case, Q0 = _case(40, 20, 12, seed=5)
    case["params"] = dict(case["params"], sgs=sgs, CI=CI)
    print(f"[gpu] faces: SGS variant sgs={sgs} CI={CI}", flush=True)
    m = orc.metrics(case)
    s = _solver(lesmi, case, Q0)
    Q = s.upload(case["Q"])
    Rg = s.download(s.residual(Q))
    Ro = orc.residual(case, m, case["Q"])
    assert (_rel(Rg, Ro) <= TOL).all(), _rel(Rg, Ro)
    Q = s.upload(case["Q"])
    dts, _ = s.advance(Q, 2, want_dt=True)
    Qg = s.download(Q)
    s.close()
    Qo = case["Q"]
    for n in range(2):
        Qo, dto, _, _ = orc.rk_step(case, m, Qo)
        assert abs(dts[n] - dto) <= 1e-14 * dto
    assert (_rel(Qg, Qo) <= TOL).all(), _rel(Qg, Qo)


def test_face_rk_steps_mixed(orc, lesmi):
    case, Q0 = _case()
    print("[gpu] faces: 2 RK steps mixed", flush=True)
    m = orc.metrics(case)
    dt = 0.8 * orc.cfl_dt(case, m, case["Q"])
    s = _solver(lesmi, case, Q0, prec=lesmi.LES_MIXED)
    Q = s.upload(case["Q"])
    Qo = case["Q"]
    for _ in range(2):
        s.rk_step(Q, dt)
        Qo, _, _, _ = orc.rk_step(case, m, Qo, dt=dt)
    q = I.interior(s.download(Q))
    qo = I.interior(Qo)
    sc = np.abs(qo).reshape(5, -1).max(1)
    sc[1:4] = sc[1:4].max()
    err = np.abs(q - qo).reshape(5, -1).max(1) / sc
    assert (err <= MIXED_BOUND).all(), err
    s.close()


def test_face_errors(lesmi):
    import torch
    case, Q0 = _case(ni=16, nj=12, nk=8)
    s = lesmi.Solver(case)
    with pytest.raises(lesmi.LesError) as e:
        s.set_face(4, lesmi.LES_FACE_EXIT, p_exit=0.7)  # k is periodic
    assert e.value.code == lesmi.LES_ERR_ARG
    with pytest.raises(lesmi.LesError):
        s.set_face(6, lesmi.LES_FACE_EXIT, p_exit=0.7)
    with pytest.raises(lesmi.LesError):
        s.set_face(1, 7)
    with pytest.raises(lesmi.LesError):
        s.set_face(1, lesmi.LES_FACE_EXIT, p_exit=0.0)
    with pytest.raises(lesmi.LesError):
        s.set_face(0, lesmi.LES_FACE_CHARACTERISTIC)  # no outside state yet
    s.close()


def _interior_rand(case, seed, scale_by_field=True):
    rng = np.random.default_rng(seed)
    a = np.zeros_like(case["Q"])
    sl = (slice(None), slice(2, -2), slice(2, -2), slice(2, -2))
    a[sl] = rng.standard_normal(a[sl].shape)
    if scale_by_field:
        a *= np.abs(I.interior(case["Q"])).reshape(5, -1).max(1)[:, None, None, None]
    return a


def _dot(a, b):
    return float((I.interior(a) * I.interior(b)).sum())


def test_face_residual_adjoint_dot_product(orc, lesmi):
    """<w, (dR/dQ) v> from the oracle's dual-number tangent (through the face
    rules of the ghost fill) against <(dR/dQ)^T w, v> from the GPU adjoint,
    which pulls the face ghosts' adjoint back to their boundary nodes."""
    case, Q0 = _case(ni=40, nj=20, nk=12)
    print("[gpu] faces: residual adjoint dot product", flush=True)
    m = orc.metrics(case)
    v = _interior_rand(case, 1)
    w = _interior_rand(case, 2, scale_by_field=False)
    _, dR = orc.residual_tangent(case, m, case["Q"], v)
    lhs = _dot(w, dR)
    s = _solver(lesmi, case, Q0)
    Qbar = s.download(s.residual_adjoint(s.upload(case["Q"]), s.upload(w)))
    rhs = _dot(Qbar, v)
    scale = float(np.abs(I.interior(w) * I.interior(dR)).sum())
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)
    s.close()


def test_face_rk_step_adjoint_dot_product(orc, lesmi):
    import torch
    case, Q0 = _case(ni=40, nj=20, nk=12)
    print("[gpu] faces: RK-step adjoint dot product", flush=True)
    m = orc.metrics(case)
    v = _interior_rand(case, 8)
    w = _interior_rand(case, 9, scale_by_field=False)
    dt = 0.8 * orc.cfl_dt(case, m, case["Q"])
    _, dQ1 = orc.rk_step_tangent(case, m, case["Q"], v, dt)
    lhs = _dot(w, dQ1)
    s = _solver(lesmi, case, Q0)
    Q = s.upload(case["Q"])
    ck = torch.empty(25 * s.fe, dtype=torch.float64, device="cuda")
    s.rk_step(Q, dt, ckpt=ck)
    Qbar = s.upload(w)
    s.adjoint_step(ck, dt, Qbar)
    rhs = _dot(s.download(Qbar), v)
    scale = float(np.abs(I.interior(w) * I.interior(dQ1)).sum())
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)
    s.close()

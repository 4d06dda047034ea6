"""The O-grid's centerline on the GPU (LES_BC_AXIS; Sec. 3) against the
oracle: cross-axis ghosts, the centerline condition, the residual next to
the axis, CFL steps in FP64 (1e-12 of each field's maximum, dt 1e-14) and
FP32-mixed (2e-6), the fused kernel against the reference kernel, a far-field
face at j-hi, the 361-azimuth grid of the paper's meshes, and the argument
errors.  J is infinite on the axis (the metrics of a collapsed face), so the
metric comparison treats those nodes apart."""
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


def _cases():
    return {"ogrid40x24x61": I.ogrid_case(40, 24, 61, seed=1),
            "ogrid24x16x361": I.ogrid_case(24, 16, 361, seed=2, CI=0.02)}


CASES = _cases()


def _rel(a, b):
    ai, bi = I.interior(a), I.interior(b)
    den = np.abs(bi).reshape(bi.shape[0], -1).max(1)
    return np.abs(ai - bi).reshape(ai.shape[0], -1).max(1) / den


@pytest.mark.parametrize("name", list(CASES))
def test_axis_metrics(orc, lesmi, name):
    case = CASES[name]
    s = lesmi.Solver(case)
    mg = s.metrics_dense()
    s.close()
    mo = orc.metrics(case)
    sl = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    a, b = mg[sl], mo[sl]
    inf_o = ~np.isfinite(b[9])
    assert inf_o.any()
    np.testing.assert_array_equal(~np.isfinite(a[9]), inf_o)  # J infinite exactly on the axis
    fin = np.isfinite(b)
    mag = np.array([np.abs(b[c][fin[c]]).max() for c in range(10)])
    den = np.array([mag[3 * (c // 3):3 * (c // 3) + 3].max() for c in range(9)] + [mag[9]])
    err = np.array([np.abs(a[c][fin[c]] - b[c][fin[c]]).max() for c in range(10)]) / den
    assert (err <= 1e-13).all(), err


@pytest.mark.parametrize("name", list(CASES))
def test_axis_residual_and_ghosts(orc, lesmi, name):
    case = CASES[name]
    print(f"[gpu] axis residual {name}", flush=True)
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    R = s.download(s.residual(Q))
    Qg = s.download(Q)
    s.close()
    m = orc.metrics(case)
    Qo = orc.fill_ghosts_faces(case, m, case["Q"])
    # ghost layers (the cross-axis rows included) as the oracle fills them;
    # the axis row holds ring means, summed in another fixed order than the
    # oracle's: within the summation bound (nk - 1) eps max|ring| per field
    off = np.ones(Qg.shape[1:], dtype=bool)
    off[:, 2, :] = False  # padded row of j = 0
    np.testing.assert_allclose(Qg[:, off], Qo[:, off], rtol=1e-15, atol=0)
    ring = np.abs(Qo[:, 2:-2, 3, 2:-2]).reshape(5, -1).max(1)
    bound = (case["nk"] - 1) * np.finfo(np.float64).eps * ring
    err = np.abs(Qg[:, :, 2, :] - Qo[:, :, 2, :]).reshape(5, -1).max(1)
    assert (err <= bound).all(), (err, bound)
    Ro = orc.residual(case, m, case["Q"])
    assert (_rel(R, Ro) <= TOL).all(), _rel(R, Ro)
    assert np.abs(I.interior(R)[:, :, 0, :]).max() == 0.0  # the axis is not advanced by R


@pytest.mark.parametrize("name", list(CASES))
def test_axis_rk_parity(orc, lesmi, name):
    case = CASES[name]
    print(f"[gpu] axis RK {name}", flush=True)
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    dts, norms = s.advance(Q, 2, want_dt=True, want_norms=True)
    Qg = s.download(Q)
    s.close()
    m = orc.metrics(case)
    Qo = case["Q"]
    for n in range(2):
        Qo, dto, no, _ = orc.rk_step(case, m, Qo)
        assert abs(dts[n] - dto) <= 1e-14 * dto, (n, dts[n], dto)
    assert np.allclose(norms, no, rtol=1e-11, atol=0)
    assert (_rel(Qg, Qo) <= TOL).all(), _rel(Qg, Qo)
    Qi = I.interior(Qg)
    nk = case["nk"]
    # every axis node is the mean of its ring, within the summation bound
    ring = Qi[:, :nk - 1, 1, :]
    bound = (nk - 1) * np.finfo(np.float64).eps * np.abs(ring).max(axis=1)[:, None, :]
    err = np.abs(Qi[:, :, 0, :] - ring.mean(axis=1)[:, None, :])
    assert (err <= bound).all(), float((err / np.maximum(bound, 1e-300)).max())


def test_axis_mixed(orc, lesmi):
    case = CASES["ogrid40x24x61"]
    s = lesmi.Solver(case, prec=lesmi.LES_MIXED)
    Q = s.upload(case["Q"])
    dts, _ = s.advance(Q, 2, want_dt=True)
    Qg = s.download(Q)
    s.close()
    m = orc.metrics(case)
    Qo = case["Q"]
    for n in range(2):
        Qo, _, _, _ = orc.rk_step(case, m, Qo, dt=dts[n])
    d = I.interior(Qg) - I.interior(Qo)
    sc = np.abs(I.interior(Qo)).reshape(5, -1).max(1)
    sc[1:4] = sc[1:4].max()
    linf = np.abs(d).reshape(5, -1).max(1) / sc
    print(f"[gpu] axis mixed: Linf {linf}", flush=True)
    assert (linf <= MIXED_BOUND).all(), linf


def test_axis_fused_matches_reference(lesmi):
    case = CASES["ogrid40x24x61"]
    out = []
    for ref in (False, True):
        s = lesmi.Solver(case)
        s.use_reference(ref)
        Q = s.upload(case["Q"])
        s.rk_step(Q, 0.0)
        out.append(s.download(Q))
        s.close()
    assert (_rel(out[0], out[1]) <= 1e-13).all(), _rel(out[0], out[1])


def test_axis_with_farfield_face(orc, lesmi):
    """The paper's radial layout: axis at j-lo, far field at j-hi."""
    case = dict(CASES["ogrid40x24x61"])
    Q0 = I.ogrid_case(40, 24, 61, seed=1, pert=0.0)["Q"]  # the unperturbed round jet outside
    rng = np.random.default_rng(9)
    Q = case["Q"].copy()
    Q[1:4, :, 3:-2] += 0.03 * rng.uniform(-1, 1, size=Q[1:4, :, 3:-2].shape)
    case["Q"] = Q
    case["faces"] = dict(types=[0, 0, 0, 3, 0, 0], p_exit=[0.0] * 6, outside=Q0)
    s = lesmi.Solver(case)
    s.set_face(3, lesmi.LES_FACE_FARFIELD, s.upload(Q0))
    Qd = s.upload(Q)
    dts, _ = s.advance(Qd, 2, want_dt=True)
    Qg = s.download(Qd)
    with pytest.raises(lesmi.LesError) as e:
        s.set_face(2, lesmi.LES_FACE_FARFIELD)  # j-lo is the axis
    assert e.value.code == lesmi.LES_ERR_ARG
    s.close()
    m = orc.metrics(case)
    Qo = Q
    for n in range(2):
        Qo, _, _, _ = orc.rk_step(case, m, Qo, dt=dts[n])
    assert (_rel(Qg, Qo) <= TOL).all(), _rel(Qg, Qo)


def test_axis_mesh_b_residual_and_dt(orc, lesmi):
    """Mesh B of Tab. 2 as an O-grid block, 256 x 128 x 361 (11.8M points),
    in the configuration the benchmark times (axis, superposed azimuthal
    seam, far-field face at the outer radius).

    The library's metrics match the oracle's to 1e-13 of each row's maximum,
    and the CFL step to 1e-14.  The residual is compared with the oracle's
    metrics handed to les_create, because at this resolution the ring next
    to the axis (J up to 1e7) makes the residual sensitive to the last bits
    of its inputs: there a metric term moved by one unit in the last place of
    its row's maximum moves R by ~1e-11 of its maximum, and a state moved by
    one unit in the last place moves the oracle's own R_rho_v by ~1.3e-12.
    So the bound per field is 1e-12 of the field's maximum, or four times the
    change that such a last-place perturbation of the state causes in the
    oracle's own residual where that is larger."""
    import torch
    case = I.ogrid_case(256, 128, 361, seed=0)
    case["faces"] = dict(types=[0, 0, 0, 3, 0, 0], p_exit=[0.0] * 6, outside=case["Q"])
    print("[gpu] axis mesh B 256x128x361 metrics, residual and dt", flush=True)
    m = orc.metrics(case)
    s = lesmi.Solver(case)
    Qd = s.upload(case["Q"])
    s.set_face(3, lesmi.LES_FACE_FARFIELD, Qd)
    dt = s.cfl_dt(Qd)
    mg = s.metrics_dense()
    s.close()
    sl = (slice(None), slice(2, -2), slice(2, -2), slice(2, -2))
    a, b = mg[sl], m[sl]
    np.testing.assert_array_equal(~np.isfinite(a[9]), ~np.isfinite(b[9]))
    fin = np.isfinite(b)
    mag = np.array([np.abs(b[c][fin[c]]).max() for c in range(10)])
    den = np.array([mag[3 * (c // 3):3 * (c // 3) + 3].max() for c in range(9)] + [mag[9]])
    err = np.array([np.abs(a[c][fin[c]] - b[c][fin[c]]).max() for c in range(10)]) / den
    assert (err <= 1e-13).all(), err
    dto = orc.cfl_dt(case, m, case["Q"])
    assert abs(dt - dto) <= 1e-14 * dto, (dt, dto)

    s = lesmi.Solver(case, metrics=torch.from_numpy(m).cuda())
    Qd = s.upload(case["Q"])
    s.set_face(3, lesmi.LES_FACE_FARFIELD, Qd)
    Rg = I.interior(s.download(s.residual(Qd)))
    s.close()
    Ro = I.interior(orc.residual(case, m, case["Q"]))
    rng = np.random.default_rng(17)
    Qp = case["Q"] * (1.0 + 2.0 ** -52 * rng.uniform(-1, 1, size=case["Q"].shape))
    Rp = I.interior(orc.residual(case, m, Qp))
    scale = np.abs(Ro).reshape(5, -1).max(1)
    floor = np.abs(Rp - Ro).reshape(5, -1).max(1) / scale
    bound = np.maximum(TOL, 4.0 * floor)
    err = np.abs(Rg - Ro).reshape(5, -1).max(1) / scale
    assert (err <= bound).all(), (err, bound)
    assert (bound <= 1e-11).all(), bound  # the floor itself stays near rounding


def test_axis_arguments(lesmi):
    case = dict(CASES["ogrid40x24x61"])
    for bc in ((3, 0, 2), (0, 3, 0), (0, 0, 3)):
        with pytest.raises(lesmi.LesError) as e:
            lesmi.Solver(dict(case, bc=bc))
        assert e.value.code == lesmi.LES_ERR_ARG


# ---------------------------------------------------------------------------
# The dynamic closure on the O-grid (R21)
# ---------------------------------------------------------------------------
DYN = {"ogrid40x24x61_dyn": lambda: I.ogrid_case(40, 24, 61, seed=1, sgs=2),
       "ogrid24x16x361_dyn_ci": lambda: I.ogrid_case(24, 16, 361, seed=2, sgs=2, CI=0.02)}


@pytest.mark.parametrize("name", list(DYN))
def test_axis_dynamic_closure(orc, lesmi, name):
    """The dynamic closure with the polar axis: the coefficients (weighted
    by the SGS fluxes they produce, as for the other blocks; the axis row,
    whose coefficients are the ring's, has zero weight), the residual and two
    CFL steps per field to 1e-12."""
    from tests.test_gpu_sgs import _column_weights
    case = DYN[name]()
    print(f"[gpu] axis dynamic closure {name}", flush=True)
    m = orc.metrics(case)
    s = lesmi.Solver(case)
    C, D = s.dynamic_coefficients(s.upload(case["Q"]))
    Co, Do = orc.dynamic_coefficients(case, m, case["Q"])
    np.testing.assert_array_equal(C[2], C[3])  # the axis column is the ring's
    with np.errstate(invalid="ignore", divide="ignore"):
        wC, wD, _ = _column_weights(orc, case, m)
    for lab, x, xo, w in (("C", C, Co, wC), ("D_T", D, Do, wD)):
        w = np.where(np.isfinite(w), w, 0.0)
        w[0] = 0.0  # the axis row
        a, ao = x[2:-2, 2:-2] * w, xo[2:-2, 2:-2] * w
        assert ao.max() > 0.0, lab
        assert np.abs(a - ao).max() <= 1e-10 * ao.max(), (lab, np.abs(a - ao).max() / ao.max())
    Qd = s.upload(case["Q"])
    Rg = s.download(s.residual(Qd))
    Ro = orc.residual(case, m, case["Q"])
    assert (_rel(Rg, Ro) <= TOL).all(), _rel(Rg, Ro)
    Qd = s.upload(case["Q"])
    dts, _ = s.advance(Qd, 2, want_dt=True)
    Qg = s.download(Qd)
    s.close()
    Qo = case["Q"]
    for n in range(2):
        Qo, dto, _, _ = orc.rk_step(case, m, Qo)
        assert abs(dts[n] - dto) <= 1e-14 * dto
    assert (_rel(Qg, Qo) <= TOL).all(), _rel(Qg, Qo)


def test_axis_dynamic_mixed_and_fused(orc, lesmi):
    """The dynamic closure on the O-grid in the FP32-mixed form (two steps
    at the FP64 steps' dt, against the oracle, to the mixed bound) and the
    fused kernel against the reference kernel."""
    case = DYN["ogrid40x24x61_dyn"]()
    m = orc.metrics(case)
    s = lesmi.Solver(case, prec=lesmi.LES_MIXED)
    Q = s.upload(case["Q"])
    dts, _ = s.advance(Q, 2, want_dt=True)
    Qg = s.download(Q)
    s.close()
    Qo = case["Q"]
    for n in range(2):
        Qo, _, _, _ = orc.rk_step(case, m, Qo, dt=dts[n])
    d = I.interior(Qg) - I.interior(Qo)
    sc = np.abs(I.interior(Qo)).reshape(5, -1).max(1)
    sc[1:4] = sc[1:4].max()
    linf = np.abs(d).reshape(5, -1).max(1) / sc
    assert (linf <= MIXED_BOUND).all(), linf
    out = []
    for ref in (False, True):
        s = lesmi.Solver(case)
        s.use_reference(ref)
        Q = s.upload(case["Q"])
        s.rk_step(Q, 0.0)
        out.append(s.download(Q))
        s.close()
    assert (_rel(out[0], out[1]) <= 1e-13).all(), _rel(out[0], out[1])


# ---------------------------------------------------------------------------
# Boundary faces around the O-grid, and the adjoint with the axis
# ---------------------------------------------------------------------------
G = I.GAMMA


def _faces_case(bc_i, seed=1):
    """The 40 x 24 x 61 O-grid with a far-field face at j-hi and, with bc_i =
    1, an entrance (i-lo) and an exit (i-hi): the paper's domain in small.
    The outside state is the unperturbed round jet."""
    case = I.ogrid_case(40, 24, 61, seed=seed)
    case["bc"] = (bc_i, 3, 2)
    Q0 = I.ogrid_case(40, 24, 61, seed=seed, pert=0.0)["Q"]
    if bc_i == 1:
        case["faces"] = dict(types=[1, 2, 0, 3, 0, 0], p_exit=[0.0, 1.0 / G, 0, 0, 0, 0], outside=Q0)
    else:
        case["faces"] = dict(types=[0, 0, 0, 3, 0, 0], p_exit=[0.0] * 6, outside=Q0)
    return case


def _solver_with_faces(lesmi, case):
    s = lesmi.Solver(case)
    fc = case["faces"]
    Q0d = s.upload(fc["outside"])
    for f, t in enumerate(fc["types"]):
        if t == 1:
            s.set_face(f, lesmi.LES_FACE_CHARACTERISTIC, Q0d)
        elif t == 2:
            s.set_face(f, lesmi.LES_FACE_EXIT, p_exit=fc["p_exit"][f])
        elif t == 3:
            s.set_face(f, lesmi.LES_FACE_FARFIELD, Q0d)
    return s


def test_axis_with_entrance_exit_and_farfield(orc, lesmi):
    """Entrance and exit faces on the axial sides of the O-grid: the ghosts of
    those sides below the axis are edges of two boundary directions and keep
    their values, as in the oracle."""
    case = _faces_case(1)
    s = _solver_with_faces(lesmi, case)
    Qd = s.upload(case["Q"])
    Rg = s.download(s.residual(Qd))
    dts, _ = s.advance(Qd, 2, want_dt=True)
    Qg = s.download(Qd)
    s.close()
    m = orc.metrics(case)
    Ro = orc.residual(case, m, case["Q"])
    assert (_rel(Rg, Ro) <= TOL).all(), _rel(Rg, Ro)
    Qo = case["Q"]
    for n in range(2):
        Qo, dto, _, _ = orc.rk_step(case, m, Qo)
        assert abs(dts[n] - dto) <= 1e-14 * dto
    assert (_rel(Qg, Qo) <= TOL).all(), _rel(Qg, Qo)


def test_axis_whole_cylinder_mixed(orc, lesmi):
    """The whole cylinder (entrance, exit, far field, axis) in the FP32-mixed
    form: two steps at the steps' own CFL dt against the FP64 oracle, to the
    mixed bound (momenta against their common scale)."""
    case = _faces_case(1)
    s = lesmi.Solver(case, prec=lesmi.LES_MIXED)
    fc = case["faces"]
    Q0d = s.upload(fc["outside"])
    s.set_face(0, lesmi.LES_FACE_CHARACTERISTIC, Q0d)
    s.set_face(1, lesmi.LES_FACE_EXIT, p_exit=fc["p_exit"][1])
    s.set_face(3, lesmi.LES_FACE_FARFIELD, Q0d)
    Qd = s.upload(case["Q"])
    dts, _ = s.advance(Qd, 2, want_dt=True)
    Qg = s.download(Qd)
    s.close()
    m = orc.metrics(case)
    Qo = case["Q"]
    for n in range(2):
        Qo, _, _, _ = orc.rk_step(case, m, Qo, dt=dts[n])
    d = I.interior(Qg) - I.interior(Qo)
    sc = np.abs(I.interior(Qo)).reshape(5, -1).max(1)
    sc[1:4] = sc[1:4].max()
    linf = np.abs(d).reshape(5, -1).max(1) / sc
    print(f"[gpu] whole cylinder mixed: Linf {linf}", flush=True)
    assert (linf <= MIXED_BOUND).all(), linf


def _noisy(case, seed):
    """Seeded 1e-4 noise on the pressure and the momenta (interior and
    ghosts), so that no pressure second difference and no velocity component
    sits on a kink of |.| where the two linearisations could take different
    branches."""
    rng = np.random.default_rng(seed)
    out = dict(case)
    Q = case["Q"].copy()
    Q[4] += 1e-4 * (1.0 / G) / (G - 1.0) * rng.uniform(-1, 1, size=Q[4].shape)
    Q[1:4] += 1e-4 * np.abs(Q[1:4]).max() * rng.uniform(-1, 1, size=Q[1:4].shape)
    out["Q"] = Q
    return out


def _adj_cases():
    return {"ogrid40x24x61": _noisy(CASES["ogrid40x24x61"], 41),
            "ogrid24x16x361_ci": _noisy(CASES["ogrid24x16x361"], 43),
            "ogrid40x24x61_farfield": _noisy(_faces_case(0), 47),
            "ogrid40x24x61_faces": _noisy(_faces_case(1), 53)}


ADJ = _adj_cases()


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


def _make(lesmi, case):
    return _solver_with_faces(lesmi, case) if "faces" in case else lesmi.Solver(case)


@pytest.mark.parametrize("name", list(ADJ))
def test_axis_residual_adjoint_dot_product(orc, lesmi, name):
    """<w, (dR/dQ) v> from the oracle's dual-number tangent against
    <(dR/dQ)^T w, v> from the GPU adjoint, with the centerline condition,
    the cross-axis ghosts, the axis limits of the eta flux and radius and the
    extrapolated fourth difference all inside dR/dQ."""
    case = ADJ[name]
    print(f"[gpu] axis residual adjoint {name}", flush=True)
    m = orc.metrics(case)
    v = _interior_rand(case, 1)
    w = _interior_rand(case, 2, scale_by_field=False)
    _, dR = orc.residual_tangent(case, m, case["Q"], v)
    lhs = _dot(w, dR)
    s = _make(lesmi, case)
    Q = s.upload(case["Q"])
    Qbar = s.download(s.residual_adjoint(Q, s.upload(w)))
    s.close()
    rhs = _dot(Qbar, v)
    scale = float(np.abs(I.interior(w) * I.interior(dR)).sum())
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)
    # nothing depends on the axis values the centerline condition overwrites
    assert np.abs(I.interior(Qbar)[:, :, 0, :]).max() == 0.0


@pytest.mark.parametrize("name,i_f", [("ogrid40x24x61", 7), ("ogrid24x16x361_ci", 5), ("ogrid40x24x61_faces", 9)])
def test_axis_rk_step_adjoint_dot_product(orc, lesmi, name, i_f):
    """One RK step with forcing on plane i_f, through the centerline condition
    of every stage input and of the result."""
    import torch
    case = ADJ[name]
    print(f"[gpu] axis rk-step adjoint {name}", flush=True)
    m = orc.metrics(case)
    rng = np.random.default_rng(7)
    f = 1e-3 * rng.uniform(-1, 1, size=(5, case["nk"], case["nj"]))
    df = rng.standard_normal(f.shape)
    v = _interior_rand(case, 8)
    w = _interior_rand(case, 9, scale_by_field=False)
    dt = 0.8 * orc.cfl_dt(case, m, case["Q"])
    _, dQ1 = orc.rk_step_tangent(case, m, case["Q"], v, dt, f=f, df=df, i_f=i_f)
    lhs = _dot(w, dQ1)
    s = _make(lesmi, case)
    s.set_forcing(torch.from_numpy(f).cuda(), i_f)
    Q = s.upload(case["Q"])
    ck = torch.empty(25 * s.fe, dtype=torch.float64, device="cuda")
    s.rk_step(Q, dt, ckpt=ck)
    Qbar = s.upload(w)
    fbar = torch.zeros(f.shape, dtype=torch.float64, device="cuda")
    s.adjoint_step(ck, dt, Qbar, fbar)
    rhs = _dot(s.download(Qbar), v) + float((fbar.cpu().numpy() * df).sum())
    s.close()
    scale = float(np.abs(I.interior(w) * I.interior(dQ1)).sum())
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)

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
    # ghost layers (the cross-axis rows included) and axis nodes as the oracle fills them
    np.testing.assert_allclose(Qg, Qo, rtol=1e-15, atol=0)
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
    np.testing.assert_allclose(Qi[:, :, 0, :], np.broadcast_to(Qi[:, :nk - 1, 1, :].mean(axis=1)[:, None, :],
                                                                 Qi[:, :, 0, :].shape), rtol=1e-14, atol=0)


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


def test_axis_arguments(lesmi):
    case = dict(CASES["ogrid40x24x61"])
    for bc in ((3, 0, 2), (0, 3, 0), (0, 0, 3)):
        with pytest.raises(lesmi.LesError) as e:
            lesmi.Solver(dict(case, bc=bc))
        assert e.value.code == lesmi.LES_ERR_ARG
    with pytest.raises(lesmi.LesError) as e:
        lesmi.Solver(dict(case, params=dict(case["params"], sgs=2)))
    assert e.value.code == lesmi.LES_ERR_ARG
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    with pytest.raises(lesmi.LesError) as e:
        s.residual_adjoint(Q, s.upload(case["Q"]))
    assert e.value.code == lesmi.LES_ERR_STATE
    s.close()

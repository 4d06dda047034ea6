"""GPU path (through the C ABI) against the FP64 CPU oracle, element by
element, on seeded inputs: metrics, residual, CFL time step, norms and RK
steps; sizes span several kernel tiles with ragged tails, plus the 32^3
Taylor-Green box (the full-size jet shard is in test_gpu_configs.py).
Tolerance: the FP64 bar of 1e-12 relative to each field's maximum; for the
Taylor-Green residual (Mach 0.1, every component a small difference of much
larger flux terms) relative to the largest component of the whole residual
vector, the reading the test states."""
import numpy as np
import pytest

from paper_2003_08746_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def lesmi():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a device"
    from paper_2003_08746_amd import lesmi as L
    L.lib()
    return L


def _rel(a, b):
    """per-field max |a - b| / max |b| over the interior"""
    ai, bi = I.interior(a), I.interior(b)
    den = np.abs(bi).reshape(bi.shape[0], -1).max(1)
    den = np.where(den == 0, 1.0, den)
    return np.abs(ai - bi).reshape(ai.shape[0], -1).max(1) / den


def _cases():
    out = {}
    out["tgv32"] = I.tgv_case(32)
    c = I.jet_case(150, 40, 20, seed=4)
    out["jet150x40x20"] = c
    n = (70, 37, 21)
    xyz = I.wavy_grid(*n, L=(2.0, 1.5, 1.0), amp=0.3)
    Q = I.smooth_state(*n, seed=9, amp=0.1)
    out["wavy70x37x21_alpha07"] = I.periodic_case(*n, xyz, Q, mu_ref=3e-3, alpha=0.7, sgs=1)
    return out


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
def test_metrics_parity(orc, lesmi, name):
    case = CASES[name]
    print(f"[gpu] metrics {name}", flush=True)
    s = lesmi.Solver(case)
    mg = s.metrics_dense()
    mo = orc.metrics(case)
    sl = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    a, b = mg[sl], mo[sl]
    # each metric term is compared with the size of its row (xi_x/J, xi_y/J,
    # xi_z/J enter the fluxes together); J with itself
    mag = np.abs(b).reshape(10, -1).max(1)
    den = np.array([mag[3 * (c // 3):3 * (c // 3) + 3].max() for c in range(9)] + [mag[9]])
    err = np.abs(a - b).reshape(10, -1).max(1) / den
    assert (err <= 1e-13).all(), err
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_residual_parity(orc, lesmi, name):
    case = CASES[name]
    print(f"[gpu] residual {name}", flush=True)
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    R, norms = s.residual(Q, want_norms=True)
    Rg = s.download(R)
    m = orc.metrics(case)
    Ro = orc.residual(case, m, case["Q"])
    err = _rel(Rg, Ro)
    if name.startswith("tgv"):
        # Mach 0.1: each residual component is ~1e-3 of the flux terms it is
        # the difference of, so FP64 rounding (~1e-16 of the fluxes) reaches
        # 1e-12 of max|R_v|; measure against the whole residual vector
        Ri, Roi_ = I.interior(Rg), I.interior(Ro)
        err = np.abs(Ri - Roi_).reshape(5, -1).max(1) / np.abs(Roi_).max()
    assert (err <= TOL).all(), err
    Roi = I.interior(Ro).reshape(5, -1)
    l2 = np.sqrt((Roi ** 2).mean(1))
    linf = np.abs(Roi).max(1)
    assert np.allclose(norms[:5], l2, rtol=1e-12, atol=0) and np.allclose(norms[5:], linf, rtol=1e-12, atol=0)
    # the interior of Q is not modified; the periodic ghosts were filled
    Qg = s.download(Q)
    assert np.array_equal(I.interior(Qg), I.interior(case["Q"]))
    assert np.array_equal(Qg, orc.fill_ghosts(case, case["Q"])) or case["bc"] != (0, 0, 0)
    s.close()


def test_caller_metrics(orc, lesmi):
    """les_create with les_metrics: the oracle's metrics handed over (no
    coordinates) give the same residual as the metrics the library computes,
    to the metrics parity bound; the library's own metrics handed back give
    the identical residual."""
    import torch
    case = CASES["wavy70x37x21_alpha07"]
    s = lesmi.Solver(case)
    R0 = s.download(s.residual(s.upload(case["Q"])))
    mine = torch.from_numpy(s.metrics_dense()).cuda()
    s.close()
    s2 = lesmi.Solver(case, metrics=mine)
    R2 = s2.download(s2.residual(s2.upload(case["Q"])))
    s2.close()
    assert np.array_equal(I.interior(R2), I.interior(R0))
    mo = torch.from_numpy(orc.metrics(case)).cuda()
    s3 = lesmi.Solver(case, metrics=mo)
    R3 = s3.download(s3.residual(s3.upload(case["Q"])))
    s3.close()
    Ro = orc.residual(case, orc.metrics(case), case["Q"])
    assert (_rel(R3, Ro) <= TOL).all(), _rel(R3, Ro)


DEGENERATE = {
    "sgs0": dict(sgs=0),                          # the paper's runs: no SGS model
    "euler": dict(sgs=0, mu_ref=0.0),             # no viscosity at all
    "k2_0": dict(k2=0.0),                         # fourth differences only
    "k4_0": dict(k4=0.0),                         # second differences only
    "no_dissipation": dict(k2=0.0, k4=0.0),
    "alpha1": dict(alpha=1.0),                    # Lambda_d = lam_d + lam_e + lam_f
}


@pytest.mark.parametrize("name", list(DEGENERATE))
def test_degenerate_parameters(orc, lesmi, name):
    """Parameter values where terms of the method vanish or its general
    branches reduce: the residual and two CFL steps against the oracle at
    the FP64 bar, on the ragged jet block."""
    base = CASES["jet150x40x20"]
    case = dict(base)
    case["params"] = dict(base["params"], **DEGENERATE[name])
    print(f"[gpu] degenerate {name}", flush=True)
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    m = orc.metrics(case)
    Rg = s.download(s.residual(Q))
    Ro = orc.residual(case, m, case["Q"])
    assert (_rel(Rg, Ro) <= TOL).all(), _rel(Rg, Ro)
    Qo = case["Q"]
    for n in range(2):
        dt, _ = s.rk_step(Q, 0.0, want_dt=True)
        Qo, dto, _, _ = orc.rk_step(case, m, Qo)
        assert abs(dt - dto) <= 1e-14 * dto, (n, dt, dto)
    assert (_rel(s.download(Q), Qo) <= TOL).all(), _rel(s.download(Q), Qo)
    s.close()


def test_residual_with_source(orc, lesmi):
    import torch
    case = CASES["jet150x40x20"]
    s = lesmi.Solver(case)
    rng = np.random.default_rng(3)
    f = rng.standard_normal((5, case["nk"], case["nj"])) * 1e-3
    s.set_forcing(torch.from_numpy(f).cuda(), 17)
    Rg = s.download(s.residual(s.upload(case["Q"])))
    Ro = orc.residual(case, orc.metrics(case), case["Q"], f=f, i_f=17)
    assert (_rel(Rg, Ro) <= TOL).all()
    s.close()


@pytest.mark.parametrize("name,steps", [("tgv32", 10), ("jet150x40x20", 3), ("wavy70x37x21_alpha07", 2)])
def test_rk_parity(orc, lesmi, name, steps):
    case = CASES[name]
    print(f"[gpu] rk {name} x{steps}", flush=True)
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    m = orc.metrics(case)
    Qo = case["Q"]
    for n in range(steps):
        dt, norms = s.rk_step(Q, 0.0, want_dt=True, want_norms=True)
        Qo, dto, no, _ = orc.rk_step(case, m, Qo)
        assert abs(dt - dto) <= 1e-14 * dto, (n, dt, dto)
        assert np.allclose(norms, no, rtol=1e-11, atol=0), (n, norms, no)
    Qg = s.download(Q)
    assert (_rel(Qg, Qo) <= TOL).all(), _rel(Qg, Qo)
    # the increment itself agrees to a tight relative bound as well
    inc = _rel(Qg - case["Q"], Qo - case["Q"])
    assert (inc <= 1e-9).all(), inc
    s.close()


def test_rk_fixed_dt_and_checkpoints(orc, lesmi):
    import torch
    case = CASES["jet150x40x20"]
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    ck = torch.zeros(5 * 5 * s.fe, dtype=torch.float64, device="cuda")
    dt = 2.5e-3
    s.rk_step(Q, dt, ckpt=ck)
    Qo, _, _, stages = orc.rk_step(case, orc.metrics(case), case["Q"], dt=dt, want_stages=True)
    assert (_rel(s.download(Q), Qo) <= TOL).all()
    for l in range(5):
        st = s.download(ck[l * 5 * s.fe:(l + 1) * 5 * s.fe])
        assert (_rel(st, stages[l]) <= TOL).all(), l
    s.close()


# ---------------------------------------------------------------------------
# GPU-side invariants, independent of the oracle
# ---------------------------------------------------------------------------
def test_gpu_freestream(lesmi):
    n = (70, 37, 21)
    xyz = I.wavy_grid(*n, L=(2.0, 1.5, 1.0), amp=0.3)
    Q = I.uniform_state((n[2] + 4, n[1] + 4, n[0] + 4), vel=(0.8, 0.8, 0.8))
    case = I.periodic_case(*n, xyz, Q, mu_ref=1e-3)
    s = lesmi.Solver(case)
    Qd = s.upload(Q)
    R = I.interior(s.download(s.residual(Qd)))
    m = I.interior(s.metrics_dense())
    # size of one flux-difference term: J |metric row| (rho |u|^2 + p)
    rows = np.maximum.reduce([np.sqrt(m[3 * d] ** 2 + m[3 * d + 1] ** 2 + m[3 * d + 2] ** 2) for d in range(3)])
    scale = float((m[9] * rows).max() * (3 * 0.8 ** 2 + 1 / I.GAMMA))
    assert np.abs(R).max() <= 1e-13 * scale
    for _ in range(5):
        s.rk_step(Qd)
    Qn = s.download(Qd)
    assert (_rel(Qn, Q) <= 1e-13).all()
    s.close()


def test_gpu_conservation(lesmi):
    case = CASES["wavy70x37x21_alpha07"]
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    invJ = 1.0 / I.interior(s.metrics_dense())[9]
    R = I.interior(s.download(s.residual(Q)))
    RJ = (R * invJ).reshape(5, -1)
    assert (np.abs(RJ.sum(1)) <= 1e-13 * np.abs(RJ).sum(1)).all()
    tot0 = (I.interior(case["Q"]) * invJ).reshape(5, -1).sum(1)
    for _ in range(5):
        s.rk_step(Q)
    tot = (I.interior(s.download(Q)) * invJ).reshape(5, -1).sum(1)
    scale = (np.abs(I.interior(case["Q"])) * invJ).reshape(5, -1).sum(1)
    assert (np.abs(tot - tot0) <= 1e-13 * scale).all()
    s.close()


def test_nonfinite_reported(lesmi):
    case = CASES["tgv32"]
    s = lesmi.Solver(case)
    Qh = case["Q"].copy()
    Qh[0, 10, 11, 12] = np.nan
    Q = s.upload(Qh)
    with pytest.raises(lesmi.LesError) as e:
        s.rk_step(Q, 0.0, want_dt=True, want_norms=True)
    assert e.value.code == lesmi.LES_ERR_NONFINITE
    # negative density is caught by the time-step reduction
    Qh = case["Q"].copy()
    Qh[0, 5, 6, 7] = -1.0
    Q = s.upload(Qh)
    with pytest.raises(lesmi.LesError) as e:
        s.cfl_dt(Q)
    assert e.value.code == lesmi.LES_ERR_NONFINITE
    # the context stays usable
    Q = s.upload(case["Q"])
    dt, _ = s.rk_step(Q, 0.0, want_dt=True)
    assert dt > 0
    s.close()


def test_argument_errors(lesmi):
    case = CASES["tgv32"]
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    with pytest.raises(lesmi.LesError) as e:
        lesmi.les_residual(s.ctx, Q.data_ptr(), Q.data_ptr())
    assert e.value.code == lesmi.LES_ERR_ARG
    with pytest.raises(lesmi.LesError) as e:
        lesmi.les_set_forcing(s.ctx, Q.data_ptr(), 99)
    assert e.value.code == lesmi.LES_ERR_ARG
    with pytest.raises(lesmi.LesError) as e:
        lesmi.les_rk_step(s.ctx, Q.data_ptr(), float("nan"))
    assert e.value.code == lesmi.LES_ERR_ARG
    # the state must be 16-byte aligned (checked before any kernel is launched)
    with pytest.raises(lesmi.LesError) as e:
        lesmi.les_rk_step(s.ctx, Q.data_ptr() + 8, 1e-3)
    assert e.value.code == lesmi.LES_ERR_ARG
    s.close()

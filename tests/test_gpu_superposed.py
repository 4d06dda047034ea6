"""Superposed periodic direction (LES_BC_PERIODIC_SUPERPOSED: the first and
last nodes coincide, as the azimuthal direction of the paper's O-grid,
Sec. 3) against the oracle, against the GPU's own plain periodic block of one
node fewer, and the adjoint (dot-product tests against the oracle's tangents).  Tolerances: 1e-12 relative to each
field's maximum (FP64), 2e-6 (mixed)."""
import numpy as np
import pytest

from paper_2003_08746_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def lesmi():
    import torch
    assert torch.cuda.is_available()
    from paper_2003_08746_amd import lesmi as L
    L.lib()
    return L


def _cases():
    n = (47, 33, 19)
    wavy = I.periodic_case(*n, I.wavy_grid(*n, L=(2.0, 1.5, 1.0), amp=0.3), I.smooth_state(*n, seed=21, amp=0.1),
                           mu_ref=3e-3, sgs=1)
    return {"wavy47x33x19_k": (wavy, 2), "jet61x29x23_i": (I.jet_case(61, 29, 23, seed=3), 0)}


def _rel(a, b):
    ai, bi = I.interior(a), I.interior(b)
    den = np.abs(bi).reshape(bi.shape[0], -1).max(1)
    return np.abs(ai - bi).reshape(ai.shape[0], -1).max(1) / den


def _along(a, axis, sl):
    idx = [slice(None)] * a.ndim
    idx[a.ndim - 1 - axis] = sl
    return a[tuple(idx)]


@pytest.mark.parametrize("name", list(_cases()))
def test_superposed_matches_oracle(orc, lesmi, name):
    base, axis = _cases()[name]
    case = I.superposed_case(base, axis)
    print(f"[gpu] superposed {name}", flush=True)
    m = orc.metrics(case)
    s = lesmi.Solver(case)
    mg = s.metrics_dense()
    b1 = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))  # nodes of [-1, n]^3
    err = np.abs(mg[b1] - m[b1]).reshape(10, -1).max(1) / np.abs(m[b1]).reshape(10, -1).max(1)
    assert (err <= 1e-13).all(), err
    Q = s.upload(case["Q"])
    R = s.residual(Q)
    Ro = orc.residual(case, m, case["Q"])
    assert (_rel(s.download(R), Ro) <= TOL).all(), _rel(s.download(R), Ro)
    dt = 0.8 * orc.cfl_dt(case, m, case["Q"])
    Qo = case["Q"]
    for _ in range(2):
        s.rk_step(Q, dt)
        Qo, _, _, _ = orc.rk_step(case, m, Qo, dt=dt)
    Qg = s.download(Q)
    assert (_rel(Qg, Qo) <= TOL).all(), _rel(Qg, Qo)
    # the superposed node still equals node 0
    n = case[("ni", "nj", "nk")[axis]]
    qi = I.interior(Qg)
    np.testing.assert_array_equal(_along(qi, axis, slice(n - 1, n)), _along(qi, axis, slice(0, 1)))
    s.close()
    # mixed precision on the same block
    sm = lesmi.Solver(case, prec=lesmi.LES_MIXED)
    Qm = sm.upload(case["Q"])
    for _ in range(2):
        sm.rk_step(Qm, dt)
    qm, qo = I.interior(sm.download(Qm)), I.interior(Qo)
    sc = np.abs(qo).reshape(5, -1).max(1)
    sc[1:4] = sc[1:4].max()
    assert (np.abs(qm - qo).reshape(5, -1).max(1) / sc <= 2e-6).all()
    sm.close()


def test_superposed_equals_periodic_on_gpu(lesmi):
    """Two GPU steps of the superposed block reproduce, on nodes 0..n-1, two
    GPU steps of the periodic block of n nodes."""
    base, axis = _cases()["jet61x29x23_i"]
    case = I.superposed_case(base, axis)
    n = base["ni"]
    a, b = lesmi.Solver(base), lesmi.Solver(case)
    Qa, Qb = a.upload(base["Q"]), b.upload(case["Q"])
    dt = a.cfl_dt(Qa)
    assert b.cfl_dt(Qb) == dt
    for _ in range(2):
        a.rk_step(Qa, dt)
        b.rk_step(Qb, dt)
    qa, qb = I.interior(a.download(Qa)), I.interior(b.download(Qb))
    d = np.abs(_along(qb, axis, slice(0, n)) - qa).reshape(5, -1).max(1) / np.abs(qa).reshape(5, -1).max(1)
    assert (d <= 1e-14).all(), d
    a.close()
    b.close()


def test_superposed_statistics(orc, lesmi):
    """Running statistics along a superposed k direction count the repeated
    plane once: the GPU sums of the superposed block equal the GPU sums of the
    periodic block of one plane fewer (the same terms in the same order), and
    the oracle's to the summation bound of the plain statistics test."""
    base, axis = _cases()["wavy47x33x19_k"]
    case = I.superposed_case(base, axis)
    print("[gpu] superposed statistics", flush=True)
    a, b = lesmi.Solver(base), lesmi.Solver(case)
    assert a.stats_planes == base["nk"] and b.stats_planes == base["nk"] == case["nk"] - 1
    acc_a = a.stats_accumulate(a.upload(base["Q"])).cpu().numpy()
    acc_b = b.stats_accumulate(b.upload(case["Q"])).cpu().numpy()
    a.close()
    b.close()
    np.testing.assert_array_equal(acc_b, acc_a)
    want = orc.stats(case, case["Q"])
    n = b.stats_planes
    eps = np.finfo(np.float64).eps
    for k in range(want.shape[0]):
        tol = (n * n + 8 * n) * eps * np.abs(want[k]).max()
        assert np.abs(acc_b[k] - want[k]).max() <= tol, (k, np.abs(acc_b[k] - want[k]).max(), tol)


def test_superposed_dynamic_closure(orc, lesmi):
    """The dynamic closure's column sums along a superposed k direction run
    over its distinct planes: the superposed block's coefficients equal the
    periodic block's of one plane fewer on the GPU, bit for bit, and its
    residual matches the oracle's to 1e-12."""
    base, axis = _cases()["wavy47x33x19_k"]
    base = dict(base, params=dict(base["params"], sgs=2))
    case = I.superposed_case(base, axis)
    print("[gpu] superposed dynamic closure", flush=True)
    a, b = lesmi.Solver(base), lesmi.Solver(case)
    Ca, Da = a.dynamic_coefficients(a.upload(base["Q"]))
    Cb, Db = b.dynamic_coefficients(b.upload(case["Q"]))
    np.testing.assert_array_equal(Cb, Ca)
    np.testing.assert_array_equal(Db, Da)
    Rg = b.download(b.residual(b.upload(case["Q"])))
    a.close()
    b.close()
    Ro = orc.residual(case, orc.metrics(case), case["Q"])
    assert (_rel(Rg, Ro) <= TOL).all(), _rel(Rg, Ro)


def test_superposed_rollout_objective(orc, lesmi):
    """The forcing workload on a block with a superposed k direction: the
    probe objective sums the plane's distinct azimuths, and its gradient with
    respect to the forcing (GPU adjoint) matches the oracle's dual-number
    directional derivative (3 steps, 2 directions)."""
    import torch
    from paper_2003_08746_amd.rollout import LesRollout
    base, axis = _cases()["wavy47x33x19_k"]
    case = I.superposed_case(base, axis)
    print("[gpu] superposed rollout objective", flush=True)
    i_f, i_p, p_inf, nsteps = 5, 12, 1.0 / I.GAMMA, 3
    f = 1e-3 * np.random.default_rng(1).uniform(-1, 1, size=(5, case["nk"], case["nj"]))
    m = orc.metrics(case)
    dt = 0.8 * orc.cfl_dt(case, m, case["Q"])
    s = lesmi.Solver(case)
    Q0 = s.upload(case["Q"])
    ft = torch.from_numpy(f).cuda().requires_grad_(True)
    J = LesRollout.apply(ft, Q0, s, nsteps, dt, i_f, i_p, p_inf, "stages")
    J.backward()
    g = ft.grad.cpu().numpy()
    s.close()
    for seed in (2, 3):
        d = np.random.default_rng(seed).standard_normal(f.shape)
        d /= np.linalg.norm(d)
        Jo, dJo = orc.objective_rollout(case, m, case["Q"], f, d, i_f, i_p, p_inf, nsteps, dt)
        assert abs(J.item() - Jo) <= 1e-11 * abs(Jo), (J.item(), Jo)
        gd = float((g * d).sum())
        assert abs(gd - dJo) <= 1e-10 * abs(dJo), (seed, gd, dJo)


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


@pytest.mark.parametrize("name", list(_cases()))
def test_superposed_adjoint_dot_products(orc, lesmi, name):
    """Residual and RK-step adjoints on a superposed block against the
    oracle's dual-number tangents (images of period n - 1 folded back)."""
    import torch
    base, axis = _cases()[name]
    if name.startswith("jet"):
        # the perfectly expanded jet has a uniform pressure, where the sensor
        # |p+ - 2p + p-| sits on its kink; seeded noise resolves the branches
        base = dict(base)
        Qn = base["Q"].copy()
        Qn[4] += 1e-4 * (1.0 / I.GAMMA) / (I.GAMMA - 1.0) * np.random.default_rng(17).uniform(-1, 1, Qn[4].shape)
        base["Q"] = Qn
    case = I.superposed_case(base, axis)
    print(f"[gpu] superposed adjoint {name}", flush=True)
    m = orc.metrics(case)
    v = _interior_rand(case, 1)
    w = _interior_rand(case, 2, scale_by_field=False)
    _, dR = orc.residual_tangent(case, m, case["Q"], v)
    s = lesmi.Solver(case)
    Qbar = s.download(s.residual_adjoint(s.upload(case["Q"]), s.upload(w)))
    lhs, rhs = _dot(w, dR), _dot(Qbar, v)
    scale = float(np.abs(I.interior(w) * I.interior(dR)).sum())
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)
    dt = 0.8 * orc.cfl_dt(case, m, case["Q"])
    _, dQ1 = orc.rk_step_tangent(case, m, case["Q"], v, dt)
    Q = s.upload(case["Q"])
    ck = torch.empty(25 * s.fe, dtype=torch.float64, device="cuda")
    s.rk_step(Q, dt, ckpt=ck)
    Qb = s.upload(w)
    s.adjoint_step(ck, dt, Qb)
    lhs, rhs = _dot(w, dQ1), _dot(s.download(Qb), v)
    scale = float(np.abs(I.interior(w) * I.interior(dQ1)).sum())
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)
    s.close()


@pytest.mark.parametrize("name", list(_cases()))
def test_superposed_adjoint_physical_directions(orc, lesmi, name):
    """The superposed block's residual adjoint along perturbations that move
    node 0 and its duplicate node n together (the directions that keep the
    block a periodic one) against the plain periodic block's oracle tangent:
    <Js^T w, v_s> = <w', Jp v>, w' = w with its plane n added onto plane 0.
    Neither side depends on how the ghosts break the tie between the two
    copies of the seam."""
    base, axis = _cases()[name]
    if name.startswith("jet"):
        base = dict(base)
        Qn = base["Q"].copy()
        Qn[4] += 1e-4 * (1.0 / I.GAMMA) / (I.GAMMA - 1.0) * np.random.default_rng(17).uniform(-1, 1, Qn[4].shape)
        base["Q"] = Qn
    case = I.superposed_case(base, axis)
    n = base[("ni", "nj", "nk")[axis]]
    print(f"[gpu] superposed adjoint, physical directions {name}", flush=True)
    v = _interior_rand(base, 3)
    vs = I.superposed_case(dict(base, Q=v), axis)["Q"]
    w = _interior_rand(case, 4, scale_by_field=False)
    wf = np.zeros_like(base["Q"])
    wi = I.interior(w)
    wfi = _along(wi, axis, slice(0, n)).copy()
    _along(wfi, axis, slice(0, 1))[...] += _along(wi, axis, slice(n, n + 1))
    wf[:, 2:-2, 2:-2, 2:-2] = wfi
    _, dRp = orc.residual_tangent(base, orc.metrics(base), base["Q"], v)
    s = lesmi.Solver(case)
    Qbar = s.download(s.residual_adjoint(s.upload(case["Q"]), s.upload(w)))
    s.close()
    lhs = _dot(Qbar, vs)
    rhs = _dot(wf, dRp)
    scale = float(np.abs(I.interior(wf) * I.interior(dRp)).sum())
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)

"""Hand-written GPU adjoint against the oracle's exact dual-number tangent
(dot-product tests <w, J v> = <J^T w, v>) and against central finite
differences of the GPU forward rollout for the forcing workload (128 x 64 x
64 jet grid, 50 steps, probe-plane pressure objective, 16 directions)."""
import numpy as np
import pytest

from paper_2003_08746_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lesmi():
    import torch
    assert torch.cuda.is_available()
    from paper_2003_08746_amd import lesmi as L
    L.lib()
    return L


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


def _with_pressure_noise(case, seed, amp=1e-4):
    """Where the pressure is uniform along a grid line (the perfectly expanded
    jet everywhere, the Taylor-Green vortex on its nodal lines) the sensor
    |p+ - 2p + p-| sits on its kink and the branch of d|x|/dx would be chosen
    by last-bit rounding (which differs between the CPU, the GPU and between
    kernels).  A seeded pressure perturbation of 1e-4 p_inf resolves every
    branch."""
    rng = np.random.default_rng(seed)
    Q = case["Q"].copy()
    Q[4] += amp * (1.0 / I.GAMMA) / (I.GAMMA - 1.0) * rng.uniform(-1, 1, size=Q[4].shape)
    out = dict(case)
    out["Q"] = Q
    return out


def _with_momentum_noise(case, seed, amp=1e-4):
    """Seeded momentum perturbation of amp times the largest momentum
    component (interior and ghosts), so that no velocity component is zero."""
    rng = np.random.default_rng(seed)
    Q = case["Q"].copy()
    scale = np.abs(Q[1:4]).max()
    Q[1:4] += amp * scale * rng.uniform(-1, 1, size=Q[1:4].shape)
    out = dict(case)
    out["Q"] = Q
    return out


def _cases():
    c1 = _with_pressure_noise(I.jet_case(61, 29, 23, seed=3), 17)
    n = (47, 33, 19)
    xyz = I.wavy_grid(*n, L=(2.0, 1.5, 1.0), amp=0.3)
    c2 = I.periodic_case(*n, xyz, I.smooth_state(*n, seed=5, amp=0.1), mu_ref=3e-3, alpha=0.7, sgs=1)
    # the Taylor-Green state sits on kinks of |.| everywhere: w = 0 at every
    # node (|U_zeta| = 0), v = 0 on whole grid lines and the pressure is
    # exactly p_inf along every line where cos 2x + cos 2y = 0 (zero second
    # difference); seeded noise on the momenta and the pressure moves it off
    # them, so that both linearisations take the same branches
    c3 = _with_momentum_noise(_with_pressure_noise(I.tgv_case(32), 19), 29)
    # the smallest block the library takes, periodic in every direction:
    # every interior node but six is within two nodes of a periodic seam, so
    # the ghost-image fold carries most of the adjoint (axes of 5, 6 and 7
    # nodes: seam bands with a core of 1, 2 and 3 nodes)
    n = (5, 6, 7)
    xyz = I.wavy_grid(*n, L=(1.0, 1.2, 1.4), amp=0.2)
    c4 = I.periodic_case(*n, xyz, I.smooth_state(*n, seed=13, amp=0.1), mu_ref=3e-3, sgs=1)
    # the isotropic SGS stress (sigma_kk / 3 added to the flux pressure)
    c5 = _with_pressure_noise(I.jet_case(61, 29, 23, seed=3, CI=0.05), 31)
    n = (47, 33, 19)
    c6 = I.periodic_case(*n, I.wavy_grid(*n, L=(2.0, 1.5, 1.0), amp=0.3), I.smooth_state(*n, seed=5, amp=0.1),
                         mu_ref=3e-3, sgs=1, CI=0.05)
    return {"jet61x29x23": c1, "wavy47x33x19_alpha07": c2, "tgv32": c3, "wavy5x6x7": c4,
            "jet61x29x23_ci": c5, "wavy47x33x19_ci": c6}


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
def test_residual_adjoint_dot_product(orc, lesmi, name):
    case = CASES[name]
    print(f"[gpu] residual adjoint {name}", flush=True)
    m = orc.metrics(case)
    v = _interior_rand(case, 1)
    w = _interior_rand(case, 2, scale_by_field=False)
    _, dR = orc.residual_tangent(case, m, case["Q"], v)
    lhs = _dot(w, dR)
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    Qbar = s.download(s.residual_adjoint(Q, s.upload(w)))
    rhs = _dot(Qbar, v)
    scale = float(np.abs(I.interior(w) * I.interior(dR)).sum())
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)
    s.close()


@pytest.mark.parametrize("name,i_f", [("jet61x29x23", 7), ("wavy5x6x7", 2), ("jet61x29x23_ci", 7)])
def test_rk_step_adjoint_dot_product(orc, lesmi, name, i_f):
    """One RK step with forcing on plane i_f: <w, dQ^{n+1}> against
    <Qbar, v> + <fbar, df>.  On the 5 x 6 x 7 periodic box the forcing plane
    i = 2 holds both nodes away from every seam and nodes next to one, so
    the source-plane update and the final sum are taken on both paths."""
    import torch
    case = CASES[name]
    print(f"[gpu] rk-step adjoint {name}", flush=True)
    m = orc.metrics(case)
    rng = np.random.default_rng(7)
    f = 1e-3 * rng.uniform(-1, 1, size=(5, case["nk"], case["nj"]))
    df = rng.standard_normal(f.shape)
    v = _interior_rand(case, 8)
    w = _interior_rand(case, 9, scale_by_field=False)
    dt = 0.8 * orc.cfl_dt(case, m, case["Q"])
    _, dQ1 = orc.rk_step_tangent(case, m, case["Q"], v, dt, f=f, df=df, i_f=i_f)
    lhs = _dot(w, dQ1)
    s = lesmi.Solver(case)
    s.set_forcing(torch.from_numpy(f).cuda(), i_f)
    Q = s.upload(case["Q"])
    ck = torch.empty(25 * s.fe, dtype=torch.float64, device="cuda")
    s.rk_step(Q, dt, ckpt=ck)
    Qbar = s.upload(w)
    fbar = torch.zeros(f.shape, dtype=torch.float64, device="cuda")
    s.adjoint_step(ck, dt, Qbar, fbar)
    rhs = _dot(s.download(Qbar), v) + float((fbar.cpu().numpy() * df).sum())
    scale = float(np.abs(I.interior(w) * I.interior(dQ1)).sum())
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)
    s.close()


def _forcing_setup(ni, nj, nk, seed_f=1):
    # jet initial state plus 1e-4 seeded pressure noise, so that the sensor's
    # branches are decided by resolved pressure differences
    case = _with_pressure_noise(I.jet_case(ni, nj, nk, seed=0), 23)
    rng = np.random.default_rng(seed_f)
    f = 1e-3 * rng.uniform(-1, 1, size=(5, nk, nj))
    return case, f


def test_rollout_gradient_vs_oracle_dual(orc, lesmi):
    """Reduced forcing workload (48 x 20 x 16, 10 steps; the oracle's dual
    numbers over the full 128 x 64 x 64 x 50-step workload would take hours
    per direction): <dJ/df, d> from the GPU adjoint against the oracle's
    dual-number directional derivative on all 16 seeded directions of the
    finite-difference check (seeds 2..17)."""
    import torch
    from paper_2003_08746_amd.rollout import LesRollout
    case, f = _forcing_setup(48, 20, 16)
    i_f, i_p, p_inf, nsteps = 8, 40, 1.0 / I.GAMMA, 10
    m = orc.metrics(case)
    dt = orc.cfl_dt(case, m, case["Q"])
    s = lesmi.Solver(case)
    Q0 = s.upload(case["Q"])
    ft = torch.from_numpy(f).cuda().requires_grad_(True)
    J = LesRollout.apply(ft, Q0, s, nsteps, dt, i_f, i_p, p_inf, "stages")
    J.backward()
    g = ft.grad.cpu().numpy()
    for seed in range(2, 18):
        d = np.random.default_rng(seed).standard_normal(f.shape)
        d /= np.linalg.norm(d)
        Jo, dJo = orc.objective_rollout(case, m, case["Q"], f, d, i_f, i_p, p_inf, nsteps, dt)
        assert abs(J.item() - Jo) <= 1e-11 * abs(Jo), (J.item(), Jo)
        gd = float((g * d).sum())
        assert abs(gd - dJo) <= 1e-10 * abs(dJo), (seed, gd, dJo)
    s.close()


def test_rollout_gradient_vs_finite_differences(lesmi):
    """Forcing workload at full size: 128 x 64 x 64 jet grid, 50 steps,
    source plane i = 8, probe plane i = 16 (a probe 32 planes downstream is
    not reached physically within 50 steps, so its sensitivity is below FP64
    resolution and finite differences return noise); 16 seeded unit
    directions."""
    import torch
    from paper_2003_08746_amd.rollout import LesRollout, objective
    case, f = _forcing_setup(128, 64, 64)
    i_f, i_p, p_inf, nsteps = 8, 16, 1.0 / I.GAMMA, 50
    s = lesmi.Solver(case)
    Q0 = s.upload(case["Q"])
    dt = s.cfl_dt(Q0)
    ft = torch.from_numpy(f).cuda().requires_grad_(True)
    J = LesRollout.apply(ft, Q0, s, nsteps, dt, i_f, i_p, p_inf, "stages")
    J.backward()
    g = ft.grad.clone()
    # recompute mode gives the same gradient
    ft2 = torch.from_numpy(f).cuda().requires_grad_(True)
    J2 = LesRollout.apply(ft2, Q0, s, nsteps, dt, i_f, i_p, p_inf, "steps")
    J2.backward()
    assert torch.equal(J.detach(), J2.detach())
    assert torch.allclose(ft2.grad, g, rtol=1e-13, atol=0)
    fscale = float(np.abs(f).max())
    gnorm = float(torch.linalg.norm(g).item())
    f_t = torch.from_numpy(f).cuda()
    errs, rel = {}, {}
    for hfac in (1e-2, 1e-3):
        h = hfac * fscale
        errs[hfac], rel[hfac] = [], []
        for seed in range(2, 18):
            d = np.random.default_rng(seed).standard_normal(f.shape)
            d /= np.linalg.norm(d)
            dt_ = torch.from_numpy(d).cuda()
            Jp = objective(s, f_t + h * dt_, Q0, nsteps, dt, i_f, i_p, p_inf)
            Jm = objective(s, f_t - h * dt_, Q0, nsteps, dt, i_f, i_p, p_inf)
            fd = (Jp - Jm) / (2 * h)
            gd = float((g * dt_).sum().item())
            # unit directions: compare with |g| |d| = |g| (a random direction
            # can make <g, d> itself arbitrarily small)
            errs[hfac].append(abs(fd - gd) / gnorm)
            rel[hfac].append(abs(fd - gd) / abs(gd))
        print(f"[gpu] h = {hfac:g} max|f|: |fd - <g,d>| / |g| max {max(errs[hfac]):.2e}; "
              f"relative to |<g,d>|: median {np.median(rel[hfac]):.2e} max {max(rel[hfac]):.2e}; "
              f"J = {J.item():.6e}, |g| = {gnorm:.3e}", flush=True)
    assert max(min(errs[1e-2][n], errs[1e-3][n]) for n in range(16)) <= 1e-6, errs
    s.close()

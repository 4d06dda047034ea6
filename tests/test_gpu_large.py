"""The 800 x 500 x 500 jet shard (2.0e8 points) in the launch configuration
the benchmark times, checked against the oracle on sampled windows.

One Runge-Kutta step of the whole shard runs on the GPU.  The oracle cannot
step 2e8 points, but a step only reaches two nodes per stage: the residual
at a node reads the state within two nodes along each axis (and one along
the edge diagonals).  So the oracle steps a 25^3 window cut out of the
initial state, with its ghost layers frozen at the initial values (every
window face is a Dirichlet face).  Stage 1 is exact on the whole window
interior; each later stage loses two more nodes next to an artificial window
face, so after five stages every node at least 8 nodes from an artificial
face is the exact full-shard result.  Where the window face is the shard's
own Dirichlet face (j = 0 or j = nj-1) the frozen ghosts are the true ones
and no node is lost.  Windows straddle the periodic seams in i and k (their
coordinates are the period-shifted images) and include the shear layer.

The same windows also check the CFL time step (the shard's global minimum is
at most every window's minimum) and the residual max-norm (at least every
window's maximum |R(Q^n)|), and the FP32-mixed path against the FP64 oracle
at its stated bound.  dt is fixed (1e-3, close to the shard's CFL step) so
that both sides take the same step.
"""
import numpy as np
import pytest

from paper_2003_08746_amd import inputs as I

from tests.windows import gather as _gather, window

pytestmark = pytest.mark.gpu

N = (800, 500, 500)  # ni, nj, nk
W = 25  # window interior points per axis
DT = 1e-3
TOL = 1e-12
MIXED_BOUND = 2e-6


@pytest.fixture(scope="module")
def lesmi():
    import torch
    assert torch.cuda.is_available()
    from paper_2003_08746_amd import lesmi as L
    L.lib()
    return L


@pytest.fixture(scope="module")
def shard():
    import torch
    print(f"[gpu] generating jet shard {N} on the device", flush=True)
    case = I.jet_case_device(*N, seed=0)
    yield case
    case.clear()
    torch.cuda.empty_cache()


def _starts(case):
    """Window interior start (i0, j0, k0) of each sample window."""
    ni, nj, nk = N
    y = case["xyz"][1, 2, 2:-2, 2].cpu().numpy()  # y along j at i = k = 0
    j_shear = int(np.argmin(np.abs(y - 0.5)))    # the upper shear layer
    rng = np.random.default_rng(5)
    r = (int(rng.integers(0, ni)), int(rng.integers(0, nj - W + 1)), int(rng.integers(0, nk)))
    return [(-12, nj // 2 - 12, -12),        # both periodic seams, centre line
            (400, 0, 250),                   # lower Dirichlet face
            (ni - 13, nj - W, nk - 12),      # upper Dirichlet face, both seams
            (100, j_shear - 12, 300),        # shear layer
            (ni // 2, j_shear - 12, nk - 3), # shear layer across the k seam
            r]


def _scale(case, share_momentum=False):
    """Per-field max |Q^n| over the whole shard interior: the scale errors are
    measured against (a window in the far field at rest has no momentum scale
    of its own)."""
    sc = case["Q"][:, 2:-2, 2:-2, 2:-2].abs().amax(dim=(1, 2, 3)).cpu().numpy()
    if share_momentum:
        sc[1:4] = sc[1:4].max()
    return sc


def _err(a, b, scale):
    return np.abs(a - b).reshape(5, -1).max(1) / scale


def test_large_shard_fp64_windows(orc, lesmi, shard):
    import torch
    case = shard
    starts = _starts(case)
    wins = [window(case, s, W) for s in starts]
    scale = _scale(case)
    print("[gpu] large shard FP64: create + one step", flush=True)
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    dt_gpu = s.cfl_dt(Q)
    _, norms = s.rk_step(Q, DT, want_norms=True)
    torch.cuda.synchronize()
    Qv = s.view(Q)
    res = []
    for (win, idx, core), st in zip(wins, starts):
        m = orc.metrics(win)
        # global CFL minimum <= this window's minimum; global max|R| >= this window's
        dt_w = orc.cfl_dt(win, m, win["Q"])
        # (1e-12: coordinates across a seam are the period-shifted images, which
        # differ from the shard's own analytic ghost coordinates in the last bits)
        assert dt_gpu <= dt_w * (1 + 1e-12), (st, dt_gpu, dt_w)
        R = I.interior(orc.residual(win, m, win["Q"]))
        assert (norms[5:] >= np.abs(R).reshape(5, -1).max(1) * (1 - 1e-12)).all(), (st, norms[5:])
        Qo, _, _, _ = orc.rk_step(win, m, win["Q"], dt=DT)
        res.append((st, _gather(Qv, *idx)[core], Qo[core], win["Q"][core]))
    # the increment Q^{n+1} - Q^n is measured against its largest value over
    # all windows (oracle side; the shear-layer windows set it): inside the
    # jet core the residual nearly cancels, and its own scale would only
    # magnify rounding
    inc_scale = np.max([np.abs(b - q0).reshape(5, -1).max(1) for _, _, b, q0 in res], axis=0)
    for st, a, b, q0 in res:
        err = _err(a, b, scale)
        inc = _err(a - q0, b - q0, inc_scale)
        print(f"[gpu] window {st}: core {a.shape[1:]} rel {err.max():.2e} increment {inc.max():.2e}", flush=True)
        assert (err <= TOL).all(), (st, err)
        assert (inc <= 1e-9).all(), (st, inc)
    s.close()
    del Q, Qv
    torch.cuda.empty_cache()


def test_large_shard_mixed_windows(orc, lesmi, shard):
    import torch
    case = shard
    starts = _starts(case)
    wins = [window(case, s, W) for s in starts]
    scale = _scale(case, share_momentum=True)
    print("[gpu] large shard mixed: create + one step", flush=True)
    s = lesmi.Solver(case, prec=lesmi.LES_MIXED)
    Q = s.upload(case["Q"])
    s.rk_step(Q, DT)
    torch.cuda.synchronize()
    Qv = s.view(Q)
    for (win, idx, core), st in zip(wins, starts):
        m = orc.metrics(win)
        Qo, _, _, _ = orc.rk_step(win, m, win["Q"], dt=DT)
        Qg = _gather(Qv, *idx)
        err = _err(Qg[core], Qo[core], scale)
        print(f"[gpu] mixed window {st}: Linf {err}", flush=True)
        assert (err <= MIXED_BOUND).all(), (st, err)
    s.close()
    del Q, Qv
    torch.cuda.empty_cache()


def test_large_shard_advance_matches_rk_steps(lesmi, shard):
    """The benchmark's timed call on the full shard: les_advance over two
    steps (the second step's dt reduced by the first step's last stage)
    equals two les_rk_step calls that take that dt from a pass of their own
    (the windows above check les_rk_step against the oracle)."""
    import torch
    case = shard
    print("[gpu] large shard: les_advance x2 against two les_rk_step calls", flush=True)
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    dts, norms = s.advance(Q, 2, want_dt=True, want_norms=True)
    Q2 = s.upload(case["Q"])
    dt0, _ = s.rk_step(Q2, 0.0, want_dt=True)
    assert abs(dt0 - dts[0]) <= 1e-15 * dt0, (dt0, dts[0])
    dt1 = s.cfl_dt(Q2)
    assert abs(dt1 - dts[1]) <= 1e-15 * dt1, (dt1, dts[1])
    _, norms2 = s.rk_step(Q2, float(dts[1]), want_norms=True)
    assert np.allclose(norms, norms2, rtol=1e-13, atol=0)
    a, b = s.view(Q)[:, 2:-2, 2:-2, 2:-2], s.view(Q2)[:, 2:-2, 2:-2, 2:-2]
    d = ((a - b).abs().reshape(5, -1).amax(1) / b.abs().reshape(5, -1).amax(1)).cpu().numpy()
    print(f"[gpu] large shard advance vs rk_step: dt {dts}, rel {d}", flush=True)
    assert (d <= 1e-15).all(), d
    s.close()
    del Q, Q2, a, b
    torch.cuda.empty_cache()

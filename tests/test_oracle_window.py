"""Locality of one Runge-Kutta step (CPU): the oracle's full-shard step on a
small jet shard equals, at every core node, the oracle's step on a window cut
out of the shard with frozen ghost layers (the argument in tests/windows.py).

This pins the stencil reach of the oracle's residual (two nodes along an
axis, one along an edge diagonal): a term that read further (or a ghost fill
that reached across the window) changes core nodes and fails here.  It also
validates the window construction used to check the GPU's large-shard step,
including windows across the periodic seams and on the Dirichlet faces.
"""
import numpy as np
import pytest

from paper_2003_08746_amd import inputs as I
from tests.windows import REACH, window

W = 21


@pytest.fixture(scope="module")
def shard_step(orc):
    case = I.jet_case(60, 48, 44, seed=2)
    m = orc.metrics(case)
    dt = 0.8 * orc.cfl_dt(case, m, case["Q"])
    Q1, _, _, _ = orc.rk_step(case, m, case["Q"], dt=dt)
    return case, dt, Q1


@pytest.mark.parametrize("start", [(-10, 13, -10), (20, 0, 5), (50, 48 - W, 40), (7, 20, 30)])
def test_window_step_equals_shard_step(orc, shard_step, start):
    case, dt, Q1 = shard_step
    win, idx, core = window(case, start, W)
    m = orc.metrics(win)
    Qw, _, _, _ = orc.rk_step(win, m, win["Q"], dt=dt)
    full = Q1[:, idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]]
    scale = np.abs(I.interior(case["Q"])).reshape(5, -1).max(1)
    err = np.abs(Qw[core] - full[core]).reshape(5, -1).max(1) / scale
    assert (err <= 1e-13).all(), (start, err)
    # control: five nodes closer to an artificial face (here the lower k face)
    # than REACH the frozen ghosts are clearly visible (the error decays about
    # tenfold per node towards the core), so the window does see them
    lo = 2 + REACH - 5
    edge = (slice(None), slice(lo, lo + 1), core[2], core[3])
    e_edge = np.abs(Qw[edge] - full[edge]).reshape(5, -1).max(1) / scale
    assert e_edge.max() > 1e-11, (start, e_edge)

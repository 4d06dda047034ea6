"""The largest block the library takes: 800 x 800 x 812, whose padded fields
hold 99.7 % of the 2^29 elements that 32-bit offsets address (a larger block
is refused at creation).  One FP64 Runge-Kutta step of the whole block on the
GPU, checked against the oracle on 25^3 windows at the far corner of the
block (the largest offsets) and across the periodic seams, as in the large
shard test."""
import numpy as np
import pytest

from paper_2003_08746_amd import inputs as I

from tests.windows import gather as _gather, window

pytestmark = pytest.mark.gpu

N = (800, 800, 812)  # ni, nj, nk
W = 25
DT = 1e-3
TOL = 1e-12


@pytest.fixture(scope="module")
def lesmi():
    import torch
    assert torch.cuda.is_available()
    from paper_2003_08746_amd import lesmi as L
    L.lib()
    return L


def test_max_block_fp64_windows(orc, lesmi):
    import torch
    L = lesmi
    assert L.les_layout_for(*N)[2] < (1 << 29)
    print(f"[gpu] generating jet block {N} on the device", flush=True)
    case = I.jet_case_device(*N, seed=1)
    ni, nj, nk = N
    starts = [(ni - W, nj - W, nk - W),      # far corner: the largest offsets
              (ni - 13, nj - W, nk - 12),    # far corner across both periodic seams
              (-12, nj // 2 - 12, nk - 12)]  # centre line across the i seam at the far k end
    wins = [window(case, st, W) for st in starts]
    sc = case["Q"][:, 2:-2, 2:-2, 2:-2].abs().amax(dim=(1, 2, 3)).cpu().numpy()
    print("[gpu] max block FP64: create + one step", flush=True)
    s = L.Solver(case)
    Q = s.upload(case["Q"])
    del case
    torch.cuda.empty_cache()
    s.rk_step(Q, DT)
    torch.cuda.synchronize()
    Qv = s.view(Q)
    for (win, idx, core), st in zip(wins, starts):
        m = orc.metrics(win)
        Qo, _, _, _ = orc.rk_step(win, m, win["Q"], dt=DT)
        a = _gather(Qv, *idx)[core]
        err = np.abs(a - Qo[core]).reshape(5, -1).max(1) / sc
        print(f"[gpu] window {st}: core {a.shape[1:]} rel {err.max():.2e}", flush=True)
        assert (err <= TOL).all(), (st, err)
    s.close()
    del Q, Qv
    torch.cuda.empty_cache()

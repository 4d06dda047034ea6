"""The paper's largest mesh on one GPU: mesh I of Tab. 2 (1700 axial x 1700
radial x 361 azimuthal points, 1.04e9 nodes) as one block, laid out as a jet
shard (periodic i and k, Dirichlet j).  Its padded fields hold about twice
the 2^29 elements that a 32-bit element offset addresses, so this runs the
stage kernel's per-segment 64-bit bases.  One FP64 Runge-Kutta step of the
whole block, checked against the oracle on 25^3 windows at the far corner of
the block (the largest offsets), across both periodic seams and across
k-chunk boundaries of the kernel's schedule, as in the large shard test.
(A window across the i seam carries the seam's period shift in its
coordinates, rounded at the scale of the period, 50: at this mesh's spacing
that moves its metrics by about 2e-13 relative, so the one window that
crosses it sits at the far corner, where the flow is quiet.)  The block
needs about 212 GB of device memory (metrics, two stage buffers and the
state), so the generator's arrays are released before each allocation."""
import numpy as np
import pytest

from paper_2003_08746_amd import inputs as I

from tests.windows import gather as _gather, window

pytestmark = pytest.mark.gpu

N = (1700, 1700, 361)  # ni, nj, nk (Tab. 2, mesh I)
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


def test_mesh_i_fp64_windows(orc, lesmi):
    import torch
    L = lesmi
    st, _, fe, _ = L.les_layout_for(*N)
    assert fe > (1 << 29)  # beyond 32-bit element offsets from the field base
    print(f"[gpu] generating jet block {N} on the device", flush=True)
    case = I.jet_case_device(*N, seed=1)
    ni, nj, nk = N
    starts = [(ni - W, nj - W, nk - W),      # far corner: the largest offsets
              (ni - 13, nj - W, nk - 12),    # far corner across both periodic seams
              (ni // 2 - 12, nj // 2 - 12, 108),  # centre line, straddling k = 122
              (ni // 2, 0, 230)]             # the j-lo face, straddling k = 244
    # (on a 256-CU device the schedule marches 61-plane k chunks: k = 122 and
    # 244 start new segments, whose bases move by whole chunks)
    wins = [window(case, st_, W) for st_ in starts]
    sc = case["Q"][:, 2:-2, 2:-2, 2:-2].abs().amax(dim=(1, 2, 3)).cpu().numpy()
    torch.cuda.empty_cache()
    print("[gpu] mesh I FP64: create", flush=True)
    s = L.Solver(case)
    case["xyz"] = None
    torch.cuda.empty_cache()
    Q = s.upload(case["Q"])
    del case
    torch.cuda.empty_cache()
    print("[gpu] mesh I FP64: one step", flush=True)
    s.rk_step(Q, DT)
    torch.cuda.synchronize()
    Qv = s.view(Q)
    for (win, idx, core), st_ in zip(wins, starts):
        m = orc.metrics(win)
        Qo, _, _, _ = orc.rk_step(win, m, win["Q"], dt=DT)
        a = _gather(Qv, *idx)[core]
        err = np.abs(a - Qo[core]).reshape(5, -1).max(1) / sc
        print(f"[gpu] window {st_}: core {a.shape[1:]} rel {err.max():.2e}", flush=True)
        assert (err <= TOL).all(), (st_, err)
    s.close()
    del Q, Qv
    torch.cuda.empty_cache()

"""The fused, LDS-tiled, k-marching stage kernel against the one-thread-per-
node reference kernel (both GPU) and against the oracle, on sizes chosen to
leave ragged tiles in i and j and chunk boundaries in k; and the
mixed-precision path against the FP64 oracle with its stated error bound."""
import os

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


def _rel(a, b):
    ai, bi = I.interior(a), I.interior(b)
    den = np.abs(bi).reshape(bi.shape[0], -1).max(1)
    den = np.where(den == 0, 1.0, den)
    return np.abs(ai - bi).reshape(ai.shape[0], -1).max(1) / den


@pytest.mark.parametrize("shape,seg", [((61, 29, 23), "5"), ((31, 15, 9), "4"), ((93, 43, 17), ""),
                                       ((40, 20, 12), "7"), ((61, 29, 23), "40"), ((93, 43, 37), "200")])
def test_fused_matches_reference_kernel(lesmi, shape, seg, monkeypatch):
    """tiles 30 x 14 in (i, j): every shape leaves a ragged last tile; the
    segment sizes (tile-planes per persistent block) put segment starts and
    ends inside k and segments that span two tiles.  A share larger than nk
    (the last two cases) switches the blocks to round-robin (chunk, tile)
    segments, the schedule of the largest shards."""
    if seg:
        monkeypatch.setenv("LES_SEG", seg)
    else:
        monkeypatch.delenv("LES_SEG", raising=False)
    chunk = seg
    ni, nj, nk = shape
    case = I.jet_case(ni, nj, nk, seed=11)
    print(f"[gpu] fused vs reference {shape} chunk={chunk or 'auto'}", flush=True)
    a = lesmi.Solver(case)
    b = lesmi.Solver(case)
    b.use_reference(True)
    Qa = a.upload(case["Q"])
    Qb = b.upload(case["Q"])
    for _ in range(2):
        dta, na = a.rk_step(Qa, 0.0, want_dt=True, want_norms=True)
        dtb, nb = b.rk_step(Qb, 0.0, want_dt=True, want_norms=True)
        assert dta == dtb or abs(dta - dtb) <= 1e-15 * dtb
        assert np.allclose(na, nb, rtol=1e-11, atol=0)
    ga, gb = a.download(Qa), b.download(Qb)
    assert (_rel(ga, gb) <= 1e-13).all(), _rel(ga, gb)
    assert (_rel(ga - case["Q"], gb - case["Q"]) <= 1e-10).all()
    a.close()
    b.close()


def test_fused_matches_oracle_periodic_odd(orc, lesmi):
    n = (47, 33, 19)
    xyz = I.wavy_grid(*n, L=(2.0, 1.5, 1.0), amp=0.3)
    Q = I.smooth_state(*n, seed=21, amp=0.1)
    case = I.periodic_case(*n, xyz, Q, mu_ref=3e-3, sgs=1)
    s = lesmi.Solver(case)
    Qd = s.upload(Q)
    m = orc.metrics(case)
    Qo = Q
    for _ in range(3):
        s.rk_step(Qd)
        Qo, _, _, _ = orc.rk_step(case, m, Qo)
    assert (_rel(s.download(Qd), Qo) <= 1e-12).all()
    s.close()


# Mixed precision (FP32 stage states, fluxes and dissipation; FP64 Q^n,
# update, metrics and reductions).  Error of Q against the FP64 oracle per
# field, relative to the field's scale: max|rho| for rho, max|e| for e and
# the largest momentum component for the three momenta (a component that
# starts at zero, like rho w in the TGV, has no scale of its own).  Bound:
# FP32 rounding (6e-8) of the stage states and of flux terms up to ~1e3
# times the residual (Mach 0.1), accumulated over the steps: 2e-6.
MIXED_BOUND = 2e-6


@pytest.mark.parametrize("name,steps", [("tgv32", 10), ("jet150x40x20", 3)])
def test_mixed_precision_error(orc, lesmi, name, steps):
    case = I.tgv_case(32) if name == "tgv32" else I.jet_case(150, 40, 20, seed=4)
    s = lesmi.Solver(case, prec=lesmi.LES_MIXED)
    Q = s.upload(case["Q"])
    m = orc.metrics(case)
    Qo = case["Q"]
    for _ in range(steps):
        dt, norms = s.rk_step(Q, 0.0, want_dt=True, want_norms=True)
        Qo, dto, no, _ = orc.rk_step(case, m, Qo)
        assert abs(dt - dto) <= 1e-6 * dto  # dt from the FP64 state
    Qg = s.download(Q)
    d = I.interior(Qg) - I.interior(Qo)
    scale = np.abs(I.interior(Qo)).reshape(5, -1).max(1)
    scale[1:4] = scale[1:4].max()
    linf = np.abs(d).reshape(5, -1).max(1) / scale
    l2 = np.sqrt((d ** 2).reshape(5, -1).mean(1)) / scale
    print(f"[gpu] mixed {name}: Linf {linf} L2 {l2}", flush=True)
    assert (linf <= MIXED_BOUND).all(), linf
    assert np.isfinite(norms).all()
    s.close()


@pytest.mark.parametrize("shape", [(61, 29, 23), (31, 15, 9)])
def test_residual_fused_matches_reference(lesmi, shape):
    """les_residual through the fused kernel (the default) against the
    reference kernel, values and norms, with a source plane."""
    import torch
    ni, nj, nk = shape
    case = I.jet_case(ni, nj, nk, seed=13)
    print(f"[gpu] residual fused vs reference {shape}", flush=True)
    f = torch.from_numpy(1e-3 * np.random.default_rng(3).uniform(-1, 1, size=(5, nk, nj))).cuda()
    out = []
    for ref in (False, True):
        s = lesmi.Solver(case)
        s.use_reference(ref)
        s.set_forcing(f, ni // 3)
        R, norms = s.residual(s.upload(case["Q"]), want_norms=True)
        out.append((s.download(R), np.asarray(norms)))
        s.close()
    (ga, na), (gb, nb) = out
    assert (_rel(ga, gb) <= 1e-13).all(), _rel(ga, gb)
    assert np.allclose(na, nb, rtol=1e-11, atol=0)

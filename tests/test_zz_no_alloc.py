"""les_residual_noalloc (the entry point for callers that cannot allocate)
against les_residual through the C ABI: residual and norms bit for bit, on
two calls in a row on the same GPU (the second on a smaller block, so that
stale partials of the first would show), plus the host-side refusal of a
context whose stage kernel runs more blocks than the scratch holds."""
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


def _compare(lesmi, case):
    import torch
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    R, norms = s.residual(Q, want_norms=True)
    R2 = s.empty_state()
    R2.fill_(7.0)  # the call must write every element it owns
    nd = torch.full((10,), -1.0, dtype=torch.float64, device="cuda")
    lesmi.les_residual_noalloc(s.ctx, Q.data_ptr(), R2.data_ptr(), nd.data_ptr())
    torch.cuda.synchronize()
    a, b = s.view(R2), s.view(R)
    assert torch.equal(a, b), float((a - b).abs().max())
    assert np.array_equal(nd.cpu().numpy(), np.asarray(norms)), (nd.cpu().numpy(), norms)
    # without norms it computes the same residual
    R3 = s.empty_state()
    lesmi.les_residual_noalloc(s.ctx, Q.data_ptr(), R3.data_ptr(), None)
    torch.cuda.synchronize()
    assert torch.equal(s.view(R3), b)
    s.close()
    return norms


def test_noalloc_matches_residual_twice(lesmi):
    big = I.jet_case(150, 40, 20, seed=4)
    small = I.jet_case(31, 15, 9, seed=13)
    print("[gpu] no-alloc residual: jet 150x40x20, then 31x15x9", flush=True)
    n1 = _compare(lesmi, big)
    n2 = _compare(lesmi, small)
    assert not np.array_equal(n1, n2)


def test_noalloc_ogrid_dynamic_closure(lesmi):
    """The no-allocation residual on an O-grid (centerline condition and
    cross-axis ghosts applied in place) with the dynamic closure (its
    coefficients formed in work arrays allocated by les_create) and a
    far-field face: bit for bit as les_residual."""
    case = I.ogrid_case(40, 24, 61, seed=1, sgs=2)
    print("[gpu] no-alloc residual: O-grid 40x24x61, dynamic closure, far field", flush=True)
    import torch
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    s.set_face(3, lesmi.LES_FACE_FARFIELD, Q)
    R, norms = s.residual(Q, want_norms=True)
    R2 = s.empty_state()
    R2.fill_(7.0)
    nd = torch.full((10,), -1.0, dtype=torch.float64, device="cuda")
    lesmi.les_residual_noalloc(s.ctx, Q.data_ptr(), R2.data_ptr(), nd.data_ptr())
    torch.cuda.synchronize()
    assert torch.equal(s.view(R2), s.view(R)), float((s.view(R2) - s.view(R)).abs().max())
    assert np.array_equal(nd.cpu().numpy(), np.asarray(norms))
    s.close()


def test_noalloc_refuses_too_many_blocks(lesmi, monkeypatch):
    import torch
    case = I.jet_case(256, 128, 128, seed=0)
    monkeypatch.setenv("LES_SEG", "1")  # one k plane per block: 11,520 blocks
    s = lesmi.Solver(case)
    monkeypatch.delenv("LES_SEG")
    Q = s.upload(case["Q"])
    R = s.empty_state()
    nd = torch.zeros(10, dtype=torch.float64, device="cuda")
    with pytest.raises(lesmi.LesError) as e:
        lesmi.les_residual_noalloc(s.ctx, Q.data_ptr(), R.data_ptr(), nd.data_ptr())
    assert e.value.code == lesmi.LES_ERR_ARG
    with pytest.raises(lesmi.LesError) as e:
        lesmi.les_residual_noalloc(s.ctx, Q.data_ptr(), R.data_ptr() + 8, nd.data_ptr())
    assert e.value.code == lesmi.LES_ERR_ARG
    s.close()

"""A run stopped, written to a restart file, read back into a new solver and
continued reproduces the uninterrupted run bit for bit (state and running
statistics), in FP64 and in the FP32-mixed mode."""
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


@pytest.mark.parametrize("prec_name", ["fp64", "mixed"])
def test_resumed_run_is_bitwise_identical(lesmi, tmp_path, prec_name):
    from paper_2003_08746_amd import restart
    prec = lesmi.LES_FP64 if prec_name == "fp64" else lesmi.LES_MIXED
    case = I.jet_case(61, 29, 23, seed=5)
    n1, n2 = 3, 3

    # uninterrupted: n1 + n2 steps, statistics after every step
    s = lesmi.Solver(case, prec=prec)
    Q = s.upload(case["Q"])
    acc = None
    t = 0.0
    for _ in range(n1 + n2):
        dt, _ = s.rk_step(Q, 0.0, want_dt=True)
        t += dt
        acc = s.stats_accumulate(Q, acc)
    ref_Q, ref_acc, ref_t = s.download(Q), acc.cpu().numpy(), t
    s.close()

    # n1 steps, restart file, new solver, n2 more steps
    s = lesmi.Solver(case, prec=prec)
    Q = s.upload(case["Q"])
    acc = None
    t = 0.0
    for _ in range(n1):
        dt, _ = s.rk_step(Q, 0.0, want_dt=True)
        t += dt
        acc = s.stats_accumulate(Q, acc)
    p = str(tmp_path / "run.safetensors")
    restart.save(p, s, Q, case, step=n1, time=t, stats=acc, samples=n1 * case["nk"])
    s.close()
    del Q, acc

    s = lesmi.Solver(case, prec=prec)
    r = restart.load(p, s, case)
    assert (r["step"], r["samples"]) == (n1, n1 * case["nk"])
    Q, acc, t = r["Q"], r["stats"], r["time"]
    for _ in range(n2):
        dt, _ = s.rk_step(Q, 0.0, want_dt=True)
        t += dt
        acc = s.stats_accumulate(Q, acc)
    got_Q, got_acc = s.download(Q), acc.cpu().numpy()
    s.close()
    assert np.array_equal(got_Q.view(np.uint64), ref_Q.view(np.uint64))
    assert np.array_equal(got_acc.view(np.uint64), ref_acc.view(np.uint64))
    assert t == ref_t

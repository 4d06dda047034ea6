"""Running flow statistics (les_stats_accumulate) against the oracle: sums
over the periodic k direction of the primitives and their second moments
(the mean-flow and RMS profiles of Sec. 6), accumulated over two states."""
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


def _cases():
    n = (5, 6, 7)
    return {
        # ragged: ni not a multiple of the 64-wide blocks, nk not of the four k ranges
        "jet61x29x23": lambda: I.jet_case(61, 29, 23, seed=3),
        "tgv32": lambda: I.tgv_case(32),
        "wavy5x6x7": lambda: I.periodic_case(*n, I.wavy_grid(*n, L=(1.0, 1.2, 1.4), amp=0.2),
                                             I.smooth_state(*n, seed=13, amp=0.1)),
        # the benchmark's jet shard
        "jet256x128x128": lambda: I.jet_case(256, 128, 128, seed=0),
    }


def _phi_max(case, Q):
    """max |phi_s| over the interior of Q, for the error bound."""
    g = case["params"]["gamma"]
    q = I.interior(Q)
    rho = q[0]
    u, v, w = q[1] / rho, q[2] / rho, q[3] / rho
    p = (g - 1.0) * (q[4] - 0.5 * rho * (u * u + v * v + w * w))
    phi = (rho, u, v, w, p, u * u, v * v, w * w, u * v, u * w, v * w, p * p)
    return np.array([np.abs(x).max() for x in phi])


@pytest.mark.parametrize("name", list(_cases()))
def test_stats_match_oracle(orc, lesmi, name):
    import torch
    case = _cases()[name]()
    print(f"[gpu] stats {name}", flush=True)
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    acc = s.stats_accumulate(Q)
    s.rk_step(Q, 0.0)  # a second, different state
    acc = s.stats_accumulate(Q, acc)
    Q1 = s.download(Q)
    torch.cuda.synchronize()
    got = acc.cpu().numpy()
    want = orc.stats(case, case["Q"])
    want = orc.stats(case, Q1, want)
    assert got.shape == want.shape == (lesmi.LES_STATS_NF, case["nj"], case["ni"])
    # each entry sums n = 2 nk terms phi_s: recursive summation in any order
    # is within (n - 1) eps sum |phi| <= n^2 eps max |phi| of the exact sum,
    # and each term carries a few ulp (u = m / rho by a reciprocal on the
    # GPU, by a division in the oracle)
    n = 2 * case["nk"]
    eps = np.finfo(np.float64).eps
    pmax = np.max([_phi_max(case, q) for q in (case["Q"], Q1)], axis=0)
    for k, f in enumerate(lesmi.STATS_FIELDS):
        tol = (n * n + 8 * n) * eps * pmax[k]
        err = np.abs(got[k] - want[k]).max()
        assert err <= tol, (f, err, tol)
    # fixed summation order: a second accumulation from zero is bitwise equal
    acc2 = s.stats_accumulate(s.upload(case["Q"]))
    acc2 = s.stats_accumulate(Q, acc2)
    assert torch.equal(acc, acc2)
    s.close()


def test_stats_profiles_uniform_flow(lesmi):
    """A uniform state: means equal the state's primitives, RMS vanish."""
    import torch
    n = (40, 9, 12)
    case = I.periodic_case(*n, I.wavy_grid(*n), np.zeros((5, n[2] + 4, n[1] + 4, n[0] + 4)))
    g = case["params"]["gamma"]
    rho, u, v, w, p = 1.3, 0.4, -0.2, 0.1, 0.8
    Q = np.zeros((5, n[2] + 4, n[1] + 4, n[0] + 4))
    Q[0], Q[1], Q[2], Q[3] = rho, rho * u, rho * v, rho * w
    Q[4] = p / (g - 1) + 0.5 * rho * (u * u + v * v + w * w)
    case["Q"] = Q
    s = lesmi.Solver(case)
    acc = None
    for _ in range(3):
        acc = s.stats_accumulate(s.upload(Q), acc)
    prof = s.stats_profiles(acc, 3 * n[2])
    for name, val in (("rho", rho), ("u", u), ("v", v), ("w", w), ("p", p)):
        assert torch.allclose(prof[name], torch.full_like(prof[name], val), rtol=1e-13, atol=0), name
    for name in ("u_rms", "v_rms", "w_rms", "p_rms"):
        assert float(prof[name].max()) <= 1e-7, name  # sqrt of a rounding-level difference
    assert float(prof["uv"].abs().max()) <= 1e-14
    s.close()


@pytest.mark.parametrize("name", ["jet61x29x23", "jet256x128x128"])
def test_stats_profiles_match_oracle(orc, lesmi, name):
    """les_stats_profiles against the oracle's profiles from the same sums
    (the oracle's, uploaded): the means are IEEE quotients on both sides, so
    they and the potential-core mask agree bit for bit; an RMS is
    sqrt(<a a> - <a>^2), whose rounding (FMA or not) moves it by at most
    sqrt(4 eps <a a>); the covariance by a few ulp of <u v> and <u><v>."""
    import torch
    case = _cases()[name]()
    print(f"[gpu] stats profiles {name}", flush=True)
    s = lesmi.Solver(case)
    Q1, _, _, _ = orc.rk_step(case, orc.metrics(case), case["Q"])
    acc = orc.stats(case, case["Q"])
    acc = orc.stats(case, Q1, acc)
    samples = 2 * case["nk"]
    u_jet = 1.4  # U_j = M_j c_inf
    cores = {}
    for frac in (0.95, 0.5):
        prof_o, core_o = orc.stats_profiles(acc, samples, u_jet, frac)
        got = s.stats_profiles(torch.from_numpy(acc).cuda(), samples, u_jet, frac)
        torch.cuda.synchronize()
        g = np.stack([got[f].cpu().numpy() for f in lesmi.PROF_FIELDS])
        assert np.array_equal(g[:5], prof_o[:5])
        assert np.array_equal(got["core"].cpu().numpy().astype(np.uint8), core_o)
        eps = np.finfo(np.float64).eps
        m = acc / samples
        for f, sq in ((5, 5), (6, 6), (7, 7), (8, 11)):
            bound = np.sqrt(4 * eps * np.abs(m[sq])) + 4 * eps * prof_o[f]
            assert (np.abs(g[f] - prof_o[f]) <= bound).all(), lesmi.PROF_FIELDS[f]
        bound = 4 * eps * (np.abs(m[8]) + np.abs(m[1] * m[2]))
        assert (np.abs(g[9] - prof_o[9]) <= bound).all()
        cores[frac] = core_o
    # the core is a real region of the jet, neither empty nor everything, and
    # the 95 % core lies inside the 50 % one
    assert 0 < cores[0.95].sum() < cores[0.5].sum() < cores[0.5].size
    assert (cores[0.95] <= cores[0.5]).all()
    with pytest.raises(lesmi.LesError) as e:
        s.stats_profiles(torch.from_numpy(acc).cuda(), 0.0)
    assert e.value.code == lesmi.LES_ERR_ARG
    with pytest.raises(lesmi.LesError) as e:
        s.stats_profiles(torch.from_numpy(acc).cuda(), samples, u_jet, 1.5)
    assert e.value.code == lesmi.LES_ERR_ARG
    s.close()

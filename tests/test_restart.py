"""Restart files (paper_2003_08746_amd/restart.py) on the host: the state
and the statistics sums round-trip bit for bit, and a file is refused for
another grid, boundary set or flow, or when it is not a restart file."""
import numpy as np
import pytest

from paper_2003_08746_amd import inputs as I
from paper_2003_08746_amd import restart


def _case():
    return I.jet_case(13, 9, 7, seed=4)


def test_round_trip_bitwise(tmp_path):
    case = _case()
    rng = np.random.default_rng(0)
    Q = rng.standard_normal((5, 7 + 4, 9 + 4, 13 + 4))
    Q[0, 0, 0, 0] = np.nextafter(1.0, 2.0)  # a value that loses its last bit in any lossy path
    S = rng.standard_normal((12, 9, 13))
    p = str(tmp_path / "r.safetensors")
    restart.write(p, Q, case, step=17, time=0.125, stats=S, samples=34)
    r = restart.read(p, case)
    assert r["Q"].dtype == np.float64 and np.array_equal(r["Q"].view(np.uint64), Q.view(np.uint64))
    assert np.array_equal(r["stats"].view(np.uint64), S.view(np.uint64))
    assert (r["step"], r["time"], r["samples"]) == (17, 0.125, 34)
    restart.write(p, Q, case)
    assert restart.read(p, case)["stats"] is None


def test_refuses_other_runs(tmp_path):
    case = _case()
    Q = np.zeros((5, 11, 13, 17))
    p = str(tmp_path / "r.safetensors")
    restart.write(p, Q, case)
    other_grid = dict(case, xyz=case["xyz"] + 1e-12)
    other_flow = dict(case, params=dict(case["params"], k4=case["params"]["k4"] * 2))
    other_bc = dict(case, bc=(0, 0, 0))
    for c in (other_grid, other_flow, other_bc):
        with pytest.raises(ValueError):
            restart.read(p, c)
    with pytest.raises(ValueError):
        restart.read(p, I.jet_case(13, 9, 8, seed=4))
    with pytest.raises(ValueError):
        restart.write(p, Q[:, 1:], case)
    with pytest.raises(ValueError):
        restart.write(p, Q.astype(np.float32), case)
    # a safetensors file that is not a restart file
    from safetensors.numpy import save_file
    q = str(tmp_path / "x.safetensors")
    save_file({"Q": Q}, q, metadata={"format": "something-else"})
    with pytest.raises(ValueError):
        restart.read(q, case)


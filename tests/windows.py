"""Windows cut out of a jet shard, for checking a full-shard Runge-Kutta step
point by point with the oracle (test helper).

A residual evaluation reads the state within two nodes of a node along each
axis (one along the edge diagonals), so one five-stage step at a node depends
on the state within ten nodes.  A window of W^3 interior nodes whose ghost
layers are frozen at Q^n (Dirichlet on every face) reproduces the full-shard
step exactly at every node at least REACH = 8 nodes from an artificial face:
stage 1 is exact on the whole window interior, and each later stage loses
two nodes next to an artificial face.  Where the window face is the shard's
own Dirichlet face the frozen ghosts are the true ones and nothing is lost.
In a periodic direction the window's coordinates are the period-shifted
images of the wrapped nodes.
"""
import numpy as np

REACH = 8


def _index(start, n, W, periodic):
    idx = np.arange(start - 2, start + W + 2)
    if periodic:
        return idx % n + 2, np.floor_divide(idx, n)
    assert idx[0] >= -2 and idx[-1] <= n + 1, (start, n)
    return idx + 2, np.zeros_like(idx)


def gather(dense, ik, ij, ii):
    """dense[:, ik, ij, ii] over the outer product of the index lists, as numpy."""
    if isinstance(dense, np.ndarray):
        return dense[:, ik[:, None, None], ij[None, :, None], ii[None, None, :]].copy()
    import torch
    dev = dense.device
    K = torch.as_tensor(ik, device=dev)[:, None, None]
    J = torch.as_tensor(ij, device=dev)[None, :, None]
    I = torch.as_tensor(ii, device=dev)[None, None, :]
    return dense[:, K, J, I].cpu().numpy()


def window(case, start, W=25):
    """(window case, index lists, core slices) for the window whose interior
    starts at node start = (i0, j0, k0) of the shard; bc of the shard must be
    (periodic, Dirichlet, periodic)."""
    assert tuple(case["bc"]) == (0, 1, 0)
    (i0, j0, k0) = start
    ni, nj, nk = case["ni"], case["nj"], case["nk"]
    ii, si = _index(i0, ni, W, True)
    ij, _ = _index(j0, nj, W, False)
    ik, sk = _index(k0, nk, W, True)
    xyz = gather(case["xyz"], ik, ij, ii)
    xyz[0] += case["period"][0] * si[None, None, :]
    xyz[2] += case["period"][2] * sk[:, None, None]
    Q = gather(case["Q"], ik, ij, ii)
    win = dict(name=f"window{start}", ni=W, nj=W, nk=W, bc=(1, 1, 1), xyz=np.ascontiguousarray(xyz),
               Q=np.ascontiguousarray(Q), params=dict(case["params"]))
    lo = [REACH] * 3
    hi = [W - REACH] * 3
    if j0 == 0:
        lo[1] = 0
    if j0 == nj - W:
        hi[1] = W
    core = (slice(None), slice(2 + lo[2], 2 + hi[2]), slice(2 + lo[1], 2 + hi[1]), slice(2 + lo[0], 2 + hi[0]))
    return win, (ik, ij, ii), core

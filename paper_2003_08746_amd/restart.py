"""Restart files: the state of a run, and its running statistics, written to
disk and read back, so that a run continues exactly where it stopped.  As
in the paper's check-points (Sec. 4: each partition writes its own solution
file, so no process waits for another), one file holds one block; the
statistics are the sums behind the mean-flow and RMS profiles of Sec. 6.

Format: one safetensors file (raw little-endian arrays behind a JSON header;
reading it executes nothing).  Tensors:
  Q      float64 (5, nk+4, nj+4, ni+4): the conserved variables of Eq. 2 on
         the padded block, ghost layers included (the Dirichlet ghosts hold
         the frozen far field that a resumed run keeps using);
  stats  float64 (LES_STATS_NF, nj, ni), optional: the running sums of
         les_stats_accumulate.
Metadata (strings): format version, ni, nj, nk, bc, step, time, the number of
statistics samples, and a SHA-256 digest of the grid coordinates, boundary
types and flow parameters.  Reading checks the digest against the caller's
case: a restart onto another grid or flow would silently be another run.

The state is copied bit for bit, and les_rk_step depends only on the state
(and the context's grid, flow and boundary settings), so a resumed run
reproduces the uninterrupted one exactly.
"""
import hashlib
import json

import numpy as np

FORMAT = "lesmi-restart-1"


def case_digest(case: dict) -> str:
    """SHA-256 of what a state is only valid with: the padded coordinates
    (host or device array), the boundary types and the flow parameters."""
    h = hashlib.sha256()
    h.update(json.dumps([int(case["ni"]), int(case["nj"]), int(case["nk"]), [int(b) for b in case["bc"]]]).encode())
    h.update(json.dumps({k: case["params"][k] for k in sorted(case["params"])}, sort_keys=True).encode())
    xyz = case["xyz"]
    if not isinstance(xyz, np.ndarray):  # torch tensor (host or device)
        xyz = xyz.detach().to("cpu").numpy()
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    flat = xyz.reshape(-1)
    step = 1 << 24
    for a in range(0, flat.size, step):
        h.update(flat[a:a + step].tobytes())
    return h.hexdigest()


def write(path: str, Q: np.ndarray, case: dict, *, step: int = 0, time: float = 0.0, stats=None,
          samples: int = 0) -> None:
    """Write a dense padded state Q (5, nk+4, nj+4, ni+4), float64, and
    optional statistics sums (host arrays) for the run described by case."""
    from safetensors.numpy import save_file
    ni, nj, nk = int(case["ni"]), int(case["nj"]), int(case["nk"])
    Q = np.ascontiguousarray(Q)
    if Q.dtype != np.float64 or Q.shape != (5, nk + 4, nj + 4, ni + 4):
        raise ValueError(f"restart: state must be float64 (5, {nk + 4}, {nj + 4}, {ni + 4}), got {Q.dtype} {Q.shape}")
    tensors = {"Q": Q}
    if stats is not None:
        stats = np.ascontiguousarray(stats)
        if stats.dtype != np.float64 or stats.ndim != 3 or stats.shape[1:] != (nj, ni):
            raise ValueError(f"restart: statistics must be float64 (n, {nj}, {ni}), got {stats.dtype} {stats.shape}")
        tensors["stats"] = stats
    meta = {"format": FORMAT, "ni": str(ni), "nj": str(nj), "nk": str(nk),
            "bc": json.dumps([int(b) for b in case["bc"]]), "step": str(int(step)), "time": repr(float(time)),
            "samples": str(int(samples)), "digest": case_digest(case)}
    save_file(tensors, path, metadata=meta)


def read(path: str, case: dict) -> dict:
    """Read a restart file written for case: dict(Q, stats (or None), step,
    time, samples), host arrays.  ValueError when the file belongs to another
    grid, boundary set or flow, or is not a restart file."""
    from safetensors import safe_open
    with safe_open(path, framework="numpy") as f:
        meta = f.metadata() or {}
        if meta.get("format") != FORMAT:
            raise ValueError(f"restart: {path} is not a {FORMAT} file")
        dims = (int(meta["ni"]), int(meta["nj"]), int(meta["nk"]))
        if dims != (int(case["ni"]), int(case["nj"]), int(case["nk"])):
            raise ValueError(f"restart: {path} holds a {dims} block, the case is "
                             f"{(case['ni'], case['nj'], case['nk'])}")
        if meta["digest"] != case_digest(case):
            raise ValueError(f"restart: {path} was written for other coordinates, boundaries or flow parameters")
        keys = set(f.keys())
        Q = f.get_tensor("Q")
        stats = f.get_tensor("stats") if "stats" in keys else None
    return dict(Q=Q, stats=stats, step=int(meta["step"]), time=float(meta["time"]), samples=int(meta["samples"]))


def save(path: str, solver, Q, case: dict, *, step: int = 0, time: float = 0.0, stats=None, samples: int = 0):
    """Write a solver's device state Q (library layout) and optional device
    statistics sums (les_stats_accumulate's array) to path."""
    write(path, solver.download(Q), case, step=step, time=time,
          stats=None if stats is None else stats.detach().to("cpu").numpy(), samples=samples)


def load(path: str, solver, case: dict) -> dict:
    """Read path back onto a solver created for case: dict(Q (device, library
    layout), stats (device or None), step, time, samples)."""
    r = read(path, case)
    t = solver.torch
    r["Q"] = solver.upload(r["Q"])
    if r["stats"] is not None:
        r["stats"] = t.from_numpy(r["stats"]).to(solver.device)
    return r

#!/usr/bin/env python3
"""Throughput of the LES Runge-Kutta hot path on one MI355X.

Workload: the 256 x 128 x 128 curvilinear jet shard (one GPU's share of the
paper's Mach 1.4, Re_D = 1.57e6 jet, Sec. 5.1), FP64, CFL 0.5.  One "step" is
one five-stage Runge-Kutta step: ghost fill, the device-side CFL time step,
five fused residual + stage-update launches, and the residual-norm
reduction (no host synchronisation inside the timed region).

Prints one JSON line:
  value      Mpoint-RK-stages/s = N * 5 * steps / wall time / 1e6 (inputs
             resident in HBM before the timed region);
  roofline   the stage kernel's algorithmic HBM bytes per launch
             (192 B per point: mean of 160 B for stage 1 and 200 B for
             stages 2-5) over its mean launch time, measured with HIP
             events around every stage launch, against 8 TB/s;
  cpu_baseline  the plain FP64 CPU oracle on a bounded sample of the same
             workload (rank 0, host cores of this machine).
Extra keys report the mixed-precision path, the adjoint/forward cost, the
shard with boundary faces (entrance, exit, far field), the running flow
statistics, the restart file (write and read rates) and the bandwidth a
plain device copy reaches (the achievable stream rate beside the 8 TB/s
peak) when those paths are available.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpoint-RK-stages/s & % HBM peak; FP32-mixed vs FP64; adjoint/forward cost"
HBM_PEAK_GBS = 8000.0
BYTES_FP64 = 192.0  # algorithmic bytes per point-stage, FP64 path
BYTES_MIXED = 168.0


def _code_only(text):
    """C++ source without comments and with whitespace collapsed: edits to
    comments or layout do not change what the stage kernel is."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_hash():
    """Hash of the stage kernel's code (the sources it is built from)."""
    h = hashlib.sha256()
    for f in ["les_stage.hip", "les_stage.hpp", "les_common.hpp"]:
        p = os.path.join(ROOT, "paper_2003_08746_amd", "csrc", f)
        if os.path.exists(p):
            h.update(_code_only(open(p).read()).encode())
    return h.hexdigest()[:16]


def load_traffic(key):
    """HBM bytes per stage launch from committed rocprofv3 counter runs, only
    if they were taken on the current stage-kernel source."""
    p = os.path.join(ROOT, "profiles", "stage_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
        e = d.get(key)
        if e and e.get("kernel_hash") == kernel_hash():
            return float(e["bytes_per_launch"])
    except Exception:
        return None
    return None


def time_gpu(case, prec, steps, warmup, setup=None):
    import torch
    from paper_2003_08746_amd import lesmi
    s = lesmi.Solver(case, prec=prec)
    Q = s.upload(case["Q"])
    if setup is not None:
        setup(s, Q)
    for _ in range(warmup):
        s.rk_step(Q)
    dt0 = s.cfl_dt(Q)  # synchronises; also checks the warmed-up state is finite
    timing = True
    if timing:
        lesmi.les_debug_stage_timing(s.ctx, True)
    stream = s.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        s.rk_step(Q)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    stage_ms, launches = (lesmi.les_debug_stage_time(s.ctx) if timing else (None, 0))
    if timing:
        lesmi.les_debug_stage_timing(s.ctx, False)
    _, norms = s.rk_step(Q, 0.0, want_norms=True)  # raises on a non-finite state
    out = dict(wall_s=wall, gpu_ms=gpu_ms, stage_ms=stage_ms, launches=launches, dt0=dt0, norms=list(norms))
    s.close()
    return out


def time_adjoint(ni=128, nj=64, nk=64, nsteps=50, i_f=8, i_p=16):
    """Forcing workload: forward rollout (stage checkpoints + probe
    objective) against the backward pass (probe adjoint + les_adjoint_step),
    both timed with HIP events on the solver's stream."""
    import numpy as np
    import torch
    from paper_2003_08746_amd import inputs, lesmi
    from paper_2003_08746_amd.rollout import LesRollout
    case = inputs.jet_case(ni, nj, nk, seed=0)
    f = torch.from_numpy(1e-3 * np.random.default_rng(1).uniform(-1, 1, size=(5, nk, nj))).cuda()
    s = lesmi.Solver(case)
    Q0 = s.upload(case["Q"])
    dt = s.cfl_dt(Q0)
    p_inf = 1.0 / inputs.GAMMA
    res = {}
    for rep in range(2):  # the first repetition warms up (allocations)
        ft = f.clone().requires_grad_(True)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        e0.record(s.stream)
        J = LesRollout.apply(ft, Q0, s, nsteps, dt, i_f, i_p, p_inf, "stages")
        e1.record(s.stream)
        J.backward()
        e2.record(s.stream)
        torch.cuda.synchronize()
        res = dict(forward_ms=e0.elapsed_time(e1), backward_ms=e1.elapsed_time(e2))
    # plain forward steps (no checkpoints, no objective) for reference
    Q = Q0.clone()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    for _ in range(nsteps):
        s.rk_step(Q, dt)
    e1.record(s.stream)
    torch.cuda.synchronize()
    plain = e0.elapsed_time(e1)
    s.close()
    return {"workload": f"jet grid {ni}x{nj}x{nk}, FP64, {nsteps} RK steps, source plane i={i_f}, probe plane i={i_p}",
            "forward_ms": round(res["forward_ms"], 3), "backward_ms": round(res["backward_ms"], 3),
            "plain_forward_ms": round(plain, 3),
            "adjoint_over_forward": round(res["backward_ms"] / res["forward_ms"], 3),
            "adjoint_over_plain_forward": round(res["backward_ms"] / plain, 3)}


def time_faces(case, steps, warmup):
    """The benchmark shard with boundary faces instead of periodic i: a
    characteristic entrance at i-lo (outside state: the initial profile), a
    subsonic exit at i-hi (ambient pressure) and characteristic far-field
    faces on both j sides; FP64, same steps as the main leg."""
    from paper_2003_08746_amd import inputs, lesmi
    c = dict(case)
    c["bc"] = (1, 1, 0)

    def setup(s, Q):
        s.set_face(0, lesmi.LES_FACE_CHARACTERISTIC, Q)
        s.set_face(1, lesmi.LES_FACE_EXIT, p_exit=1.0 / inputs.GAMMA)
        s.set_face(2, lesmi.LES_FACE_CHARACTERISTIC)
        s.set_face(3, lesmi.LES_FACE_CHARACTERISTIC)

    r = time_gpu(c, lesmi.LES_FP64, steps, warmup, setup)
    npts = case["ni"] * case["nj"] * case["nk"]
    return {"value": round(npts * 5 * steps / r["wall_s"] / 1e6, 2), "unit": "Mpoint-RK-stages/s",
            "ms_per_step": round(r["wall_s"] * 1e3 / steps, 4),
            "faces": "i-lo characteristic, i-hi exit, j-lo/j-hi characteristic, k periodic"}


def time_stats(case, calls=50):
    """Running flow statistics (les_stats_accumulate) on the benchmark shard:
    mean time per call from HIP events on the solver's stream, against its
    algorithmic bytes (Q read once, 40 B per point, plus the read-modify-write
    of the 12 column sums, 192 B per (i, j) column)."""
    import torch
    from paper_2003_08746_amd import lesmi
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    acc = s.stats_accumulate(Q)  # warm-up (allocates acc)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(s.stream)
    for _ in range(calls):
        s.stats_accumulate(Q, acc)
    ev1.record(s.stream)
    torch.cuda.synchronize()
    us = ev0.elapsed_time(ev1) * 1e3 / calls
    ni, nj, nk = case["ni"], case["nj"], case["nk"]
    byts = 40.0 * ni * nj * nk + 192.0 * ni * nj
    s.close()
    return {"us_per_call": round(us, 2), "algorithmic_GBps": round(byts / us / 1e3, 1),
            "frac_of_hbm_peak": round(byts / us / 1e3 / HBM_PEAK_GBS, 4)}


def time_copy(mib=1024, reps=10):
    """Achievable stream bandwidth on this GPU: a plain device-to-device copy
    of mib MiB, read + write bytes over the mean copy time (HIP events on the
    copy's stream), by the library's copy kernel and by torch's."""
    import torch
    from paper_2003_08746_amd import lesmi
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    out = {"bytes_moved": 2 * n * 8}
    for name, run in (("GBps", lambda: lesmi.les_debug_stream_copy(src.data_ptr(), dst.data_ptr(), n * 8,
                                                                    stream.cuda_stream)),
                      ("torch_copy_GBps", lambda: dst.copy_(src))):
        run()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(reps):
            run()
        ev1.record(stream)
        torch.cuda.synchronize()
        s = ev0.elapsed_time(ev1) / 1e3 / reps
        out[name] = round(2 * n * 8 / s / 1e9, 1)
    out["frac_of_hbm_peak"] = round(out["GBps"] / HBM_PEAK_GBS, 4)
    del src, dst
    torch.cuda.empty_cache()
    return out


def time_restart(case):
    """Restart file of the benchmark shard (state with ghosts, 5 padded FP64
    fields, plus the statistics sums): wall time to write it (device to file)
    and to read it back (file to device), in a temporary directory."""
    import tempfile
    import torch
    from paper_2003_08746_amd import lesmi, restart
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    acc = s.stats_accumulate(Q)
    nbytes = 5 * 8 * (case["ni"] + 4) * (case["nj"] + 4) * (case["nk"] + 4) + acc.numel() * 8
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "run.safetensors")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        restart.save(p, s, Q, case, step=1, time=0.0, stats=acc, samples=case["nk"])
        tw = time.perf_counter() - t0
        t0 = time.perf_counter()
        r = restart.load(p, s, case)
        torch.cuda.synchronize()
        tr = time.perf_counter() - t0
        same = bool(torch.equal(s.view(r["Q"]), s.view(Q)) and torch.equal(r["stats"], acc))
    s.close()
    return {"bytes": int(nbytes), "write_s": round(tw, 3), "read_s": round(tr, 3),
            "write_GBps": round(nbytes / tw / 1e9, 2), "read_GBps": round(nbytes / tr / 1e9, 2), "bitwise": same}


def time_large(steps, ni=800, nj=500, nk=500):
    """The 800 x 500 x 500 shard (2.0e8 points), generated on the device."""
    import torch
    from paper_2003_08746_amd import inputs, lesmi
    case = inputs.jet_case_device(ni, nj, nk, seed=0)
    npts = ni * nj * nk
    out = {"workload": f"jet shard {ni}x{nj}x{nk} ({npts:.3g} points)"}
    for name, prec, byts in (("fp64", lesmi.LES_FP64, BYTES_FP64), ("mixed", lesmi.LES_MIXED, BYTES_MIXED)):
        r = time_gpu(case, prec, steps, 1)
        v = npts * 5 * steps / r["wall_s"] / 1e6
        o = {"value": round(v, 2), "unit": "Mpoint-RK-stages/s", "ms_per_step": round(r["wall_s"] * 1e3 / steps, 3),
             "algorithmic_GBps": round(byts * npts * 5 * steps / r["wall_s"] / 1e9, 1)}
        if r["stage_ms"]:
            o["avg_stage_launch_us"] = round(r["stage_ms"] / r["launches"] * 1e3, 1)
        out[name] = o
        torch.cuda.empty_cache()
    del case
    torch.cuda.empty_cache()
    return out


def cpu_baseline(case, target_s=10.0, max_steps=3):
    import oracle
    m = oracle.metrics(case)
    Q = case["Q"]
    n = case["ni"] * case["nj"] * case["nk"]
    t0 = time.perf_counter()
    done = 0
    while done < max_steps:
        Q, _, _, _ = oracle.rk_step(case, m, Q)
        done += 1
        if time.perf_counter() - t0 >= target_s:
            break
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return dict(value=n * 5 * done / el / 1e6, unit="Mpoint-RK-stages/s", cores=cores, kind="oracle",
                sample=f"{done} RK step(s) ({done * 5} stages) of the {case['ni']}x{case['nj']}x{case['nk']} "
                       f"jet shard, FP64, {el:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--ni", type=int, default=256)
    ap.add_argument("--nj", type=int, default=128)
    ap.add_argument("--nk", type=int, default=128)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the mixed-precision, adjoint, boundary-face, statistics, restart and copy legs")
    ap.add_argument("--large", action="store_true",
                    help="also time the 800 x 500 x 500 shard (FP64 and mixed, 20 steps each)")
    ap.add_argument("--large-steps", type=int, default=20)
    ap.add_argument("--copy-kernel", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB, 5 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_kernel:
        import torch
        n = args.copy_kernel * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_kernel_bytes_read": n * 8, "copy_kernel_bytes_written": n * 8, "launches": 5}))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the residual/RK path runs on one GPU's share of the domain "
              "(multi-GPU halo exchange is not part of this build); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2003_08746_amd import inputs, lesmi
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    case = inputs.jet_case(args.ni, args.nj, args.nk, seed=0)
    npts = args.ni * args.nj * args.nk
    print(f"[bench] workload jet {args.ni}x{args.nj}x{args.nk} FP64 warmup {args.warmup} steps {args.steps}",
          file=sys.stderr, flush=True)
    r = time_gpu(case, lesmi.LES_FP64, args.steps, args.warmup)
    value = npts * 5 * args.steps / r["wall_s"] / 1e6
    ms_per_step = r["wall_s"] * 1e3 / args.steps
    avg_launch_s = r["stage_ms"] / r["launches"] / 1e3
    bytes_per_launch = BYTES_FP64 * npts
    achieved = bytes_per_launch / avg_launch_s / 1e9
    traffic = load_traffic("jet_fp64")
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mpoint-RK-stages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"jet shard {args.ni}x{args.nj}x{args.nk}, curvilinear (tanh-clustered, wavy), "
                               "Mach 1.4, Re_D 1.57e6, Smagorinsky SGS on, CFL 0.5, FP64",
                   "points": npts, "stages_per_step": 5},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / avg_launch_s / 1e9, 1),
                     "kernel": "stage (fused residual + RK update)",
                     "avg_launch_us": round(avg_launch_s * 1e6, 2),
                     "algorithmic_bytes_per_launch": int(bytes_per_launch)},
        "gpu_event_ms_per_step": round(r["gpu_ms"] / args.steps, 4),
    }
    if not args.no_extra:
        extra = {}
        try:
            rm = time_gpu(case, lesmi.LES_MIXED, args.steps, args.warmup)
            vm = npts * 5 * args.steps / rm["wall_s"] / 1e6
            extra["mixed"] = {"value": round(vm, 2), "unit": "Mpoint-RK-stages/s",
                              "speedup_vs_fp64": round(vm / value, 3),
                              "algorithmic_GBps": round(BYTES_MIXED * npts * 5 * args.steps / rm["wall_s"] / 1e9, 1)}
        except Exception as e:  # the path reports its own error; the FP64 line stands
            extra["mixed"] = {"error": str(e)[:200]}
        try:
            extra["adjoint"] = time_adjoint()
        except Exception as e:
            extra["adjoint"] = {"error": str(e)[:200]}
        try:
            extra["faces"] = time_faces(case, args.steps, args.warmup)
            extra["faces"]["vs_main"] = round(extra["faces"]["value"] / value, 3)
        except Exception as e:
            extra["faces"] = {"error": str(e)[:200]}
        try:
            extra["stats"] = time_stats(case)
        except Exception as e:
            extra["stats"] = {"error": str(e)[:200]}
        try:
            extra["restart"] = time_restart(case)
        except Exception as e:
            extra["restart"] = {"error": str(e)[:200]}
        try:
            extra["copy"] = time_copy()
            extra["copy"]["stage_frac_of_copy"] = round(achieved / extra["copy"]["GBps"], 4)
        except Exception as e:
            extra["copy"] = {"error": str(e)[:200]}
        out["extra"] = extra
    if args.large:
        out.setdefault("extra", {})["large"] = time_large(args.large_steps)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

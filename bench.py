#!/usr/bin/env python3
"""Throughput of the LES Runge-Kutta hot path on one MI355X.

Workload (headline): the 800 x 500 x 500 curvilinear jet shard (2.0e8
points, about 1e9 unknowns; the largest of the benchmark shapes, one GPU's
share of the paper's Mach 1.4, Re_D = 1.57e6 jet, Sec. 5.1), FP64, CFL 0.5,
generated on the device.  One "step" is one five-stage Runge-Kutta step:
ghost fill, five fused residual + stage-update launches (the last one also
reduces the next step's CFL time step) and the norm / time-step
reductions; the timed region is one les_advance call of K steps (no host
synchronisation inside it).

Prints one JSON line:
  value      Mpoint-RK-stages/s = N * 5 * steps / wall time / 1e6 (inputs
             resident in HBM before the timed region);
  roofline   the stage kernel's algorithmic HBM bytes per launch
             (192 B per point: mean of 160 B for stage 1 and 200 B for
             stages 2-5) over its mean launch time, measured with HIP
             events recorded on the library's stream around every stage
             launch, against 8 TB/s; traffic = HBM bytes per launch from the
             committed rocprofv3 counter runs of the same kernel source;
  cpu_baseline  the plain FP64 CPU oracle on a bounded sample of the same
             workload family (all host cores, and one thread).
Extra keys: the FP32-mixed path on the same shard (speedup and its per-field
error against the FP64 GPU path after the same steps), the 256 x 128 x 128
jet shard in FP64 and mixed, the adjoint/forward cost on the forcing
workload, the shard with boundary faces (entrance, exit, far field), the
running flow statistics, the restart file and a plain device copy (the
achievable stream rate beside the 8 TB/s peak).
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
# mixed path, a step of les_advance after its first: stage 1 reads the FP32
# copy of Q^n that the step before wrote 20 + Q^n FP64 as Q^(0) 40 + metrics
# 80 + writes the FP32 stage state 20 = 160; stages 2-4: FP32 state 20 +
# Q^(0) 40 + metrics 80 + FP32 write 20 = 160; stage 5: 20 + 40 + 80 + FP64
# write 40 + FP32 copy 20 = 200; mean 168
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


def time_gpu(case, prec, steps, warmup, setup=None, keep_state=False):
    """Warm-up, then `steps` CFL steps in one les_advance call between two
    device synchronisations; stage-kernel launches timed with HIP events on
    the library's stream."""
    import torch
    from paper_2003_08746_amd import lesmi
    s = lesmi.Solver(case, prec=prec)
    Q = s.upload(case["Q"])
    if setup is not None:
        setup(s, Q)
    if warmup:
        s.advance(Q, warmup)
    dt0 = s.cfl_dt(Q)  # synchronises; also checks the warmed-up state is finite
    lesmi.les_debug_stage_timing(s.ctx, True)
    stream = s.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    s.advance(Q, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    stage_ms, launches = lesmi.les_debug_stage_time(s.ctx)
    lesmi.les_debug_stage_timing(s.ctx, False)
    out = dict(wall_s=wall, gpu_ms=gpu_ms, stage_ms=stage_ms, launches=launches, dt0=dt0)
    if keep_state:
        out["state"] = s.view(Q).clone()
    _, norms = s.rk_step(Q, 0.0, want_norms=True)  # raises on a non-finite state
    out["norms"] = list(norms)
    s.close()
    del Q
    torch.cuda.empty_cache()
    return out


def field_errors(a, b):
    """Per-field Linf and L2 of a - b over the interior (dense padded torch
    arrays), relative to the field's max |b| (the three momenta share the
    largest momentum's scale)."""
    import torch
    d = (a - b)[:, 2:-2, 2:-2, 2:-2].reshape(5, -1)
    sc = b[:, 2:-2, 2:-2, 2:-2].abs().reshape(5, -1).amax(1)
    sc[1:4] = sc[1:4].max()
    linf = (d.abs().amax(1) / sc).cpu().tolist()
    l2 = (torch.sqrt((d * d).mean(1)) / sc).cpu().tolist()
    names = ("rho", "rho_u", "rho_v", "rho_w", "e")
    return {"linf": {n: float(f"{x:.3e}") for n, x in zip(names, linf)},
            "l2": {n: float(f"{x:.3e}") for n, x in zip(names, l2)}}


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
    """The jet shard with boundary faces instead of periodic i: a
    characteristic entrance at i-lo (outside state: the initial profile), a
    subsonic exit at i-hi (ambient pressure) and far-field faces on both j
    sides; FP64, same steps as the shard's own leg."""
    from paper_2003_08746_amd import inputs, lesmi
    c = dict(case)
    c["bc"] = (1, 1, 0)

    def setup(s, Q):
        s.set_face(0, lesmi.LES_FACE_CHARACTERISTIC, Q)
        s.set_face(1, lesmi.LES_FACE_EXIT, p_exit=1.0 / inputs.GAMMA)
        s.set_face(2, lesmi.LES_FACE_FARFIELD)
        s.set_face(3, lesmi.LES_FACE_FARFIELD)

    r = time_gpu(c, lesmi.LES_FP64, steps, warmup, setup)
    npts = case["ni"] * case["nj"] * case["nk"]
    return {"value": round(npts * 5 * steps / r["wall_s"] / 1e6, 2), "unit": "Mpoint-RK-stages/s",
            "ms_per_step": round(r["wall_s"] * 1e3 / steps, 4),
            "faces": "i-lo characteristic entrance, i-hi exit, j-lo/j-hi far field, k periodic"}


def time_variant(case, steps, warmup, what, setup=None, base=None):
    """One FP64 les_advance leg of a model or domain variant: throughput,
    step time, mean stage-kernel launch, and (with base, a dict of the same
    block's default-model leg) its ratio to that leg."""
    from paper_2003_08746_amd import lesmi
    r = time_gpu(case, lesmi.LES_FP64, steps, warmup, setup)
    npts = case["ni"] * case["nj"] * case["nk"]
    out = {"workload": what, "points": npts, "value": round(npts * 5 * steps / r["wall_s"] / 1e6, 2),
           "unit": "Mpoint-RK-stages/s", "ms_per_step": round(r["wall_s"] * 1e3 / steps, 4),
           "avg_stage_launch_us": round(r["stage_ms"] / r["launches"] * 1e3, 2)}
    if base and "value" in base:
        out["vs_default_model"] = round(out["value"] / base["value"], 3)
    return out


def time_sgs_variants(case, steps, warmup, base):
    """The 256 x 128 x 128 shard with the optional SGS models: the dynamic
    closure (five streaming kernels before every residual, the stage kernel's
    EXT instantiation) and Yoshizawa's isotropic SGS stress with the static
    model."""
    dyn = dict(case)
    dyn["params"] = dict(case["params"], sgs=2)
    ci = dict(case)
    ci["params"] = dict(case["params"], sgs=1, CI=0.05)
    return {"dynamic": time_variant(dyn, steps, warmup, "jet shard 256x128x128, dynamic closure", base=base),
            "sigma_kk": time_variant(ci, steps, warmup, "jet shard 256x128x128, Smagorinsky + sigma_kk (CI 0.05)",
                                     base=base)}


def time_ogrid(steps=20, warmup=2):
    """Mesh B of Tab. 2 as an O-grid block (256 axial x 128 radial x 361
    azimuthal points, 11.8M): the polar axis with its centerline condition,
    the superposed azimuthal seam, a far-field face at the outer radius,
    periodic axial direction."""
    from paper_2003_08746_amd import inputs, lesmi
    case = inputs.ogrid_case(256, 128, 361, seed=0)

    def setup(s, Q):
        s.set_face(3, lesmi.LES_FACE_FARFIELD, Q)

    return time_variant(case, steps, warmup, "mesh B of Tab. 2 as an O-grid 256x128x361 (axis, far field), FP64",
                        setup=setup)


def time_ogrid_adjoint(ni=128, nj=64, nk=121, reps=3):
    """One RK step with stage checkpoints and its adjoint (les_adjoint_step)
    on an O-grid block with the polar axis, the superposed azimuthal seam
    and a far-field face at the outer radius (the paper's domain; the
    adjoint then runs the centerline transpose and the face rule's
    Jacobian): forward and backward times from HIP events on the solver's
    stream, the last of reps repetitions."""
    import numpy as np
    import torch
    from paper_2003_08746_amd import inputs, lesmi
    case = inputs.ogrid_case(ni, nj, nk, seed=0)
    s = lesmi.Solver(case)
    Q = s.upload(case["Q"])
    s.set_face(3, lesmi.LES_FACE_FARFIELD, Q)
    dt = 0.5 * s.cfl_dt(Q)
    ck = torch.empty(25 * s.fe, dtype=torch.float64, device="cuda")
    w = np.zeros_like(case["Q"])
    w[:, 2:-2, 2:-2, 2:-2] = 1e-3
    Qbar0 = s.upload(w)
    res = {}
    for _ in range(reps):
        Qd = Q.clone()
        Qbar = Qbar0.clone()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        e0.record(s.stream)
        s.rk_step(Qd, dt, ckpt=ck)
        e1.record(s.stream)
        s.adjoint_step(ck, dt, Qbar)
        e2.record(s.stream)
        torch.cuda.synchronize()
        res = dict(forward_ms=round(e0.elapsed_time(e1), 4), backward_ms=round(e1.elapsed_time(e2), 4))
    s.close()
    res["adjoint_over_forward"] = round(res["backward_ms"] / res["forward_ms"], 3)
    return {"workload": f"O-grid {ni}x{nj}x{nk} (axis, superposed seam, far field), FP64, one RK step", **res}


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


def time_mesh_i(steps=3, warmup=1):
    """The paper's largest mesh, mesh I of Tab. 2 (1700 x 1700 x 361 =
    1.04e9 points), as one jet block on one GPU in FP64 (about 212 GB of
    device memory: the generator's arrays are released before each
    allocation)."""
    import torch
    from paper_2003_08746_amd import inputs, lesmi
    ni, nj, nk = 1700, 1700, 361
    torch.cuda.empty_cache()
    case = inputs.jet_case_device(ni, nj, nk, seed=0)
    torch.cuda.empty_cache()
    s = lesmi.Solver(case)
    case["xyz"] = None
    torch.cuda.empty_cache()
    Q = s.upload(case["Q"])
    del case
    torch.cuda.empty_cache()
    try:
        s.advance(Q, warmup)
        s.cfl_dt(Q)
        lesmi.les_debug_stage_timing(s.ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.advance(Q, steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stage_ms, launches = lesmi.les_debug_stage_time(s.ctx)
        lesmi.les_debug_stage_timing(s.ctx, False)
        s.rk_step(Q, 0.0, want_norms=True)  # raises on a non-finite state
    finally:
        s.close()
        del Q
        torch.cuda.empty_cache()
    npts = ni * nj * nk
    launch_s = stage_ms / launches / 1e3
    return dict(workload=f"mesh I of Tab. 2 as one jet block {ni}x{nj}x{nk}, FP64", points=npts, steps=steps,
                value=round(npts * 5 * steps / wall / 1e6, 2), unit="Mpoint-RK-stages/s",
                ms_per_step=round(wall * 1e3 / steps, 2), avg_stage_launch_us=round(launch_s * 1e6, 1),
                stage_frac_of_hbm_peak=round(BYTES_FP64 * npts / launch_s / 1e9 / HBM_PEAK_GBS, 4))


def time_shard(case, steps, warmup, label):
    """FP64 and mixed legs of one jet shard: throughput, stage-kernel launch
    time and algorithmic bandwidth, mixed speedup and the mixed path's
    per-field error against the FP64 path after the same steps."""
    from paper_2003_08746_amd import lesmi
    npts = case["ni"] * case["nj"] * case["nk"]
    out = {"workload": label}
    states = {}
    for name, prec, byts in (("fp64", lesmi.LES_FP64, BYTES_FP64), ("mixed", lesmi.LES_MIXED, BYTES_MIXED)):
        print(f"[bench] {label}: {name}, warmup {warmup}, steps {steps}", file=sys.stderr, flush=True)
        r = time_gpu(case, prec, steps, warmup, keep_state=True)
        states[name] = r.pop("state")
        v = npts * 5 * steps / r["wall_s"] / 1e6
        launch_s = r["stage_ms"] / r["launches"] / 1e3
        out[name] = {"value": round(v, 2), "unit": "Mpoint-RK-stages/s",
                     "ms_per_step": round(r["wall_s"] * 1e3 / steps, 4),
                     "gpu_event_ms_per_step": round(r["gpu_ms"] / steps, 4),
                     "avg_stage_launch_us": round(launch_s * 1e6, 2),
                     "stage_algorithmic_GBps": round(byts * npts / launch_s / 1e9, 1),
                     "stage_frac_of_hbm_peak": round(byts * npts / launch_s / 1e9 / HBM_PEAK_GBS, 4),
                     "_wall_s": r["wall_s"], "_launch_s": launch_s}
    out["mixed"]["speedup_vs_fp64"] = round(out["mixed"]["value"] / out["fp64"]["value"], 3)
    out["mixed"]["error_vs_fp64_after_steps"] = field_errors(states["mixed"], states["fp64"])
    del states
    return out


def cpu_baseline(label, n_omp=(160, 100, 100), n_one=(64, 40, 40), target_s=10.0, max_steps=5):
    """The plain FP64 oracle on bounded samples of the workload family: all
    host cores (OpenMP over k) on an n_omp block and one thread on an n_one
    block, whole RK steps until target_s."""
    import oracle
    from paper_2003_08746_amd import inputs
    avail = len(os.sched_getaffinity(0))
    legs = {}
    for name, n, threads in (("omp", n_omp, avail), ("one", n_one, 1)):
        case = inputs.jet_case(*n, seed=0)
        m = oracle.metrics(case)
        used = oracle.threads(threads)
        Q = case["Q"]
        npts = n[0] * n[1] * n[2]
        t0 = time.perf_counter()
        done = 0
        while done < max_steps:
            Q, _, _, _ = oracle.rk_step(case, m, Q)
            done += 1
            if time.perf_counter() - t0 >= target_s:
                break
        el = time.perf_counter() - t0
        legs[name] = dict(value=npts * 5 * done / el / 1e6, cores=used,
                          sample=f"{done} RK step(s) of a {n[0]}x{n[1]}x{n[2]} block of the jet grid family, "
                                 f"FP64, {el:.1f} s, {used} thread(s)")
    oracle.threads(avail)
    o = legs["omp"]
    return dict(value=round(o["value"], 4), unit="Mpoint-RK-stages/s", cores=o["cores"], kind="oracle",
                sample=o["sample"] + f" (same per-point work as the {label})",
                single_thread={"value": round(legs["one"]["value"], 4), "unit": "Mpoint-RK-stages/s",
                               "cores": 1, "sample": legs["one"]["sample"]})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--ni", type=int, default=800)
    ap.add_argument("--nj", type=int, default=500)
    ap.add_argument("--nk", type=int, default=500)
    ap.add_argument("--small-steps", type=int, default=100, help="steps of the 256 x 128 x 128 shard legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip every leg but the headline (mixed, small shard, adjoint, faces, SGS variants, "
                         "O-grid and its adjoint, statistics, restart, copy, mesh I)")
    ap.add_argument("--copy-kernel", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB, 5 times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.copy_kernel:
        import torch
        from paper_2003_08746_amd import lesmi
        n = args.copy_kernel * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            lesmi.les_debug_stream_copy(src.data_ptr(), dst.data_ptr(), n * 8, torch.cuda.current_stream().cuda_stream)
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
    ni, nj, nk = args.ni, args.nj, args.nk
    npts = ni * nj * nk
    label = f"jet shard {ni}x{nj}x{nk}"
    print(f"[bench] generating {label} on the device", file=sys.stderr, flush=True)
    case = inputs.jet_case_device(ni, nj, nk, seed=0)
    do_extra = not args.no_extra
    if do_extra:
        big = time_shard(case, args.steps, args.warmup, label)
        main_r = big["fp64"]
        wall_s, launch_s, gpu_ms = main_r.pop("_wall_s"), main_r.pop("_launch_s"), main_r["gpu_event_ms_per_step"]
        big["mixed"].pop("_wall_s"), big["mixed"].pop("_launch_s")
    else:
        print(f"[bench] {label}: fp64, warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
        r = time_gpu(case, lesmi.LES_FP64, args.steps, args.warmup)
        wall_s, launch_s, gpu_ms = r["wall_s"], r["stage_ms"] / r["launches"] / 1e3, r["gpu_ms"] / args.steps
    del case
    torch.cuda.empty_cache()
    value = npts * 5 * args.steps / wall_s / 1e6
    bytes_per_launch = BYTES_FP64 * npts
    achieved = bytes_per_launch / launch_s / 1e9
    traffic = load_traffic(f"jet{ni}x{nj}x{nk}_fp64")
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mpoint-RK-stages/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_s * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{label}, curvilinear (tanh-clustered, wavy), Mach 1.4, Re_D 1.57e6, "
                               "Smagorinsky SGS on, CFL 0.5, FP64",
                   "points": npts, "stages_per_step": 5},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic / launch_s / 1e9, 1),
                     "kernel": "stage (fused residual + RK update)",
                     "avg_launch_us": round(launch_s * 1e6, 2),
                     "algorithmic_bytes_per_launch": int(bytes_per_launch)},
        "gpu_event_ms_per_step": round(gpu_ms, 4),
    }
    if do_extra:
        extra = {"mixed": big["mixed"]}
        small = inputs.jet_case(256, 128, 128, seed=0)
        try:
            extra["jet256x128x128"] = time_shard(small, args.small_steps, 5, "jet shard 256x128x128")
            for k in ("fp64", "mixed"):
                extra["jet256x128x128"][k].pop("_wall_s"), extra["jet256x128x128"][k].pop("_launch_s")
            t_small = load_traffic("jet256x128x128_fp64")
            if t_small is not None:
                ls = extra["jet256x128x128"]["fp64"]["avg_stage_launch_us"] / 1e6
                extra["jet256x128x128"]["fp64"]["traffic_GBps"] = round(t_small / ls / 1e9, 1)
        except Exception as e:  # the leg reports its own error; the headline stands
            extra["jet256x128x128"] = {"error": str(e)[:200]}
        base = extra.get("jet256x128x128", {}).get("fp64")
        for key, fn in (("adjoint", time_adjoint),
                        ("faces", lambda: time_faces(small, args.small_steps, 5)),
                        ("sgs_variants", lambda: time_sgs_variants(small, 20, 2, base)),
                        ("ogrid", time_ogrid),
                        ("ogrid_adjoint", time_ogrid_adjoint),
                        ("stats", lambda: time_stats(small)),
                        ("restart", lambda: time_restart(small)),
                        ("copy", time_copy),
                        ("mesh_i", time_mesh_i)):
            print(f"[bench] extra: {key}", file=sys.stderr, flush=True)
            try:
                extra[key] = fn()
            except Exception as e:
                extra[key] = {"error": str(e)[:200]}
        if "value" in extra.get("faces", {}) and "fp64" in extra.get("jet256x128x128", {}):
            extra["faces"]["vs_periodic_shard"] = round(extra["faces"]["value"] /
                                                        extra["jet256x128x128"]["fp64"]["value"], 3)
        if "GBps" in extra.get("copy", {}):
            extra["copy"]["stage_frac_of_copy"] = round(achieved / extra["copy"]["GBps"], 4)
        out["extra"] = extra
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(label)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Throughput of the FDTD leapfrog (arXiv 2401.07416, section 2.1) on one
MI355X: Gcell-steps/s of the whole step (both half-steps with the fused
detection records, FP64 flux and norm sums) on the 512x512x1024 synthetic
surface-diffraction grid, FP32 state.  Prints one JSON line.

A step is eq. (9) then eq. (8) over the whole grid, with the flux partials,
every 50 steps the record plane with Q, naive norm and plane sums, and the
fixed-order FP64 finalisation; the step driver runs them as two-step sweeps
(two steps per pass over ping-pong buffers) where the grid fits one, else
as one-pass steps or in-place half-steps.  Inputs are resident in HBM
before the timed region starts.

roofline: the dominant kernel is the launch kind that takes most of the
timed region (the two-step sweep by default; the one-pass step or the
half-step kernels when selected); its algorithmic bytes per launch are 20 B
per cell in FP32, 40 B in FP64 (read R, I, V once, write R, I once: two
steps for the sweep, one for the one-pass step; 16 / 32 B for a half-step),
divided by its average launch time measured with HIP events around each
launch inside the timed region, on the stream the kernels run on.  Launches
that also write a detection record are timed apart and reported beside it.
traffic: calibrated rocprofv3 FETCH_SIZE + WRITE_SIZE per launch from
profiles/, while the kernel sources and tile match.  The FP64 legs carry
the same block for their own dominant kernel.  cpu_baseline: the FP64
oracle on this host's physical cores (OMP_PROC_BIND=close, in a child
process that never touches the GPU) on the 256x256x512 surface grid, 200
timed steps after 10 warm-up steps, with a one-core leg and the 64^3 free
packet in full beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FDTD Gcell-steps/s & %HBM roofline (FP32/FP64); batched & adjoint vs plain"
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2000)
    p.add_argument("--warmup", type=int, default=100)
    p.add_argument("--workload", default="headline")
    p.add_argument("--precision", default="f32", choices=["f32", "f64"])
    p.add_argument("--tile", default=None,
                   help='JSON dict of Sim.set_tile keywords (default: tuned table)')
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-secondary", action="store_true",
                   help="skip the FP64, adjoint and batched measurements")
    p.add_argument("--cpu-steps", type=int, default=200,
                   help="timed oracle steps on the 256x256x512 grid (after 10 warm-up steps)")
    p.add_argument("--cpu-serial-steps", type=int, default=20,
                   help="timed one-core oracle steps on the same grid (after 1 warm-up step)")
    p.add_argument("--cpu-child", action="store_true", help=argparse.SUPPRESS)
    p.add_argument("--no-timing", action="store_true",
                   help="do not bracket launches with events (value only)")
    p.add_argument("--only", default=None, choices=sorted(SECONDARIES),
                   help="run only this one secondary measurement and print its JSON (for profiling)")
    p.add_argument("--copy-probe", action="store_true",
                   help="run only a plain device copy of 1 GiB five times (calibrates the "
                        "FETCH_SIZE / WRITE_SIZE counters against known bytes)")
    return p.parse_args()


KERNEL_SOURCES = ("kernels.hpp", "dispatch.hpp", "fused.hpp", "fused_f32.hip", "fused_f64.hip", "fused2.hpp",
                  "fused2_f32.hip", "fused2_f64.hip",
                  "half_f32_w4.hip", "half_f32_w2.hip", "half_f32_w1.hip", "half_f64_w2.hip",
                  "half_f64_w1.hip")


def kernel_src_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2401_07416_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(workload_name, precision, kind, tile):
    """HBM bytes per launch of the dominant kernel from the committed PMC
    summary, scaled by the copy-kernel calibration; null if the kernel
    source or the tile changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload_name}_{precision}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_src_sha") != kernel_src_sha():
        return None
    if any(tile.get(k) != v for k, v in t.get("tile", {"missing": True}).items()):
        return None
    return float(t["hbm_bytes_per_launch"])


CPU_SHARE = 16   # host cores one GPU of the box may use


def host_cpu():
    """lscpu facts of this host and the physical cores of this process's
    affinity mask."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=30).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
                             "CPU(s)"):
                info[k.strip()] = v.strip()
    except Exception as e:  # context only
        info["error"] = repr(e)
    cpus = sorted(os.sched_getaffinity(0))
    phys = len(cpus)
    try:
        out = subprocess.run(["lscpu", "-p=CPU,CORE,SOCKET"], capture_output=True, text=True,
                             timeout=30).stdout
        core_of = {}
        for line in out.splitlines():
            if line and not line.startswith("#"):
                c, core, sock = line.split(",")[:3]
                core_of[int(c)] = (sock, core)
        phys = len({core_of.get(c, ("?", c)) for c in cpus})
    except Exception:
        pass
    info["cpus_in_affinity"] = len(cpus)
    info["physical_cores_in_affinity"] = phys
    return info, phys


def cpu_child(a):
    """The oracle timings (run in a child process whose OpenMP runtime was
    started with OMP_PROC_BIND=close): prints one JSON line."""
    import numpy as np

    import oracle
    from paper_2401_07416_amd import workloads

    def setup(w):
        g = oracle.Grid(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.hbar, w.mass, bc=w.bc)
        if w.atoms is not None and len(w.atoms):
            V = oracle.potential(g, w.atoms, soft=w.soft, cutoff=w.cutoff, kappa=w.kappa, a0=w.a0,
                                 screened=w.screened)
        else:
            V = np.zeros(g.shape)
        dt = w.dt_frac * w.hbar / oracle.emax(g, V)
        W = oracle.cap_quadratic(w.nz, *w.cap) if w.cap else None
        k0 = (np.array(w.k0, dtype=np.float64) if w.k0 is not None
              else oracle.wavevector(w.energy, w.hbar, w.mass) * np.array(w.k_dir))
        R, I = oracle.init_gaussian(g, w.r0, k0, w.sigma, dt)
        s = oracle.Sim(g, V, R, I, dt, W=W, k_det=w.k_det)
        return s

    def timed(s, warm, steps):
        s.step(warm)
        t0 = time.perf_counter()
        s.step(steps)
        return time.perf_counter() - t0

    threads = oracle.get_threads()
    out = {"threads": threads}
    w = workloads.c2_surface()
    s = setup(w)
    el = timed(s, 10, a.cpu_steps)
    out["c2"] = {"cells": w.cells, "steps": a.cpu_steps, "warmup": 10, "s": el}
    oracle.set_threads(1)
    el1 = timed(s, 1, a.cpu_serial_steps)
    out["c2_serial"] = {"cells": w.cells, "steps": a.cpu_serial_steps, "warmup": 1, "s": el1}
    oracle.set_threads(threads)
    del s
    w1 = workloads.c1_free_gaussian()
    s1 = setup(w1)
    el = timed(s1, 0, w1.steps)
    out["c1"] = {"cells": w1.cells, "steps": w1.steps, "warmup": 0, "s": el}
    print(json.dumps(out), flush=True)


def cpu_baseline(a, gpu_value, gpu_fp64_c2):
    """Time the FP64 oracle on this host: all physical cores of the
    process's affinity mask (at most the 16-core share of one GPU) with
    OMP_PROC_BIND=close on the 256x256x512 surface grid, one core on the
    same grid, and the 64^3 free packet in full."""
    import subprocess
    info, phys = host_cpu()
    threads = max(1, min(phys, CPU_SHARE))
    env = dict(os.environ, OMP_PROC_BIND="close", OMP_PLACES="cores", OMP_NUM_THREADS=str(threads))
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-child", "--cpu-steps", str(a.cpu_steps),
           "--cpu-serial-steps", str(a.cpu_serial_steps)]
    r = subprocess.run(cmd, env=env, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"oracle child failed ({r.returncode}): {r.stderr[-2000:]}")
    t = json.loads(r.stdout.strip().splitlines()[-1])

    def rate(x):
        cs = x["cells"] * x["steps"]
        return cs / x["s"] / 1e9, x["s"] / cs * 1e9

    v, ns = rate(t["c2"])
    v1, ns1 = rate(t["c2_serial"])
    vc1, nsc1 = rate(t["c1"])
    out = {"value": round(v, 4), "unit": "Gcell-steps/s", "cores": t["threads"], "kind": "oracle",
           "sample": (f"FP64 oracle on the surface-256x256x512 grid (the surface-diffraction "
                      f"workload at its 256x256x512 size), {t['c2']['steps']} timed steps after "
                      f"{t['c2']['warmup']} warm-up steps, {t['c2']['s']:.1f} s, "
                      f"{t['threads']} threads bound with OMP_PROC_BIND=close, OMP_PLACES=cores"),
           "ns_per_cell_step": round(ns, 4), "host": info,
           "single_core": {"value": round(v1, 5), "cores": 1, "steps": t["c2_serial"]["steps"],
                           "s": round(t["c2_serial"]["s"], 2), "ns_per_cell_step": round(ns1, 3)},
           "c1_free_gaussian_64cubed": {"value": round(vc1, 4), "cores": t["threads"],
                                        "steps": t["c1"]["steps"], "s": round(t["c1"]["s"], 3),
                                        "ns_per_cell_step": round(nsc1, 4),
                                        "note": "2 MB per array: cache-resident"},
           "speedup_gpu_over_cpu": round(gpu_value / v, 1),
           "speedup_note": "headline FP32 value over the FP64 oracle on all cores"}
    if gpu_fp64_c2:
        out["speedup_gpu_fp64_over_cpu_same_grid"] = round(gpu_fp64_c2 / v, 1)
        out["speedup_gpu_fp64_over_single_core_same_grid"] = round(gpu_fp64_c2 / v1, 1)
    out["paper_context"] = {
        "gpu_over_serial_cpu": 350, "gpu_over_multicore_cpu": 5.5,
        "hardware": "Quadro K620 vs one core of a 1.6 GHz Xeon E5-2603 v3, and vs 16 two-thread "
                    "Xeon Gold 6242 cores; precision not stated",
        "ns_per_cell_step": {"k620": 6, "serial": 2000, "multicore": 30}}
    return out


# algorithmic words per cell of one launch: a half-step reads the stencil
# array, the updated array and V and writes the updated array (4 words); the
# one-pass step reads R, I, V and writes R, I (5 words, one step); the
# two-step sweep moves the same 5 words for two steps
WORDS = {"half_i": 4, "half_r": 4, "fused": 5, "two_step": 5}
STEPS_PER_LAUNCH = {"half_i": 0.5, "half_r": 0.5, "fused": 1, "two_step": 2}
# a step of the two-pass form is both half-steps (8 words)
WORDS_PER_CELL_STEP = {"half_i": 8, "half_r": 8, "fused": 5, "two_step": 2.5}
KERNEL_NAMES = {"half_i": "half_step eq.(9) imaginary", "half_r": "half_step eq.(8) real",
                "fused": "fused_step eqs.(9)+(8) one-pass",
                "two_step": "fused2 two-step sweep eqs.(9)+(8)+(9)+(8)"}


def roofline_of(kt, cells, prec, workload_name, tile):
    """Roofline block of the dominant launch kind of a split timing read
    (kinds without a record; those with one are reported apart)."""
    es = 8 if prec == "f64" else 4
    plain = {k: v for k, v in kt.items() if not k.endswith("_rec")}
    dom = max(plain, key=lambda k: plain[k][0])
    tot_ms, launches = plain[dom]
    if not launches:
        return None
    avg = tot_ms / launches
    alg_bytes = WORDS[dom] * es * cells
    achieved = alg_bytes / (avg * 1e-3) / 1e9
    traffic = traffic_from_profiles(workload_name, prec, dom, tile)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": KERNEL_NAMES[dom], "avg_launch_ms": round(avg, 5),
            "alg_bytes_per_launch": alg_bytes,
            "alg_bytes_per_cell_step": WORDS_PER_CELL_STEP[dom] * es,
            "launches": {k: v[1] for k, v in kt.items()},
            "kernel_ms": {k: round(v[0], 3) for k, v in kt.items()}}
    rec = kt.get(dom + "_rec")
    if rec and rec[1]:
        ravg = rec[0] / rec[1]
        roof["record_launch_avg_ms"] = round(ravg, 5)
    if traffic is not None:
        # the memory-side rate: counted bytes per launch over this run's
        # average launch time
        roof["traffic_gbs"] = round(traffic / (avg * 1e-3) / 1e9, 1)
        roof["traffic_frac"] = round(traffic / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return roof


def record_cost(sim, w, intervals=4):
    """Cost of the detection record (eq. (15)) on the two-step plan: a
    window of whole record intervals timed launch by launch, the launches
    that write a record against those that do not."""
    h = w.record_every
    sim.timing_read_split()
    sim.set_timing(True)
    sim.step(intervals * h)
    sim.set_timing(False)
    kt = sim.timing_read_split()
    plain = {k: v for k, v in kt.items() if not k.endswith("_rec") and v[1]}
    dom = max(plain, key=lambda k: plain[k][0])
    rec = kt[dom + "_rec"]
    if not rec[1]:
        return None
    pavg = plain[dom][0] / plain[dom][1]
    ravg = rec[0] / rec[1]
    launches_per_interval = h / STEPS_PER_LAUNCH[dom]
    return {"record_every": h, "kernel": KERNEL_NAMES[dom], "record_launches": rec[1],
            "plain_launches": plain[dom][1], "record_launch_avg_ms": round(ravg, 5),
            "plain_launch_avg_ms": round(pavg, 5),
            "extra_ms_per_record": round(ravg - pavg, 5),
            "overhead_frac_of_interval": round((ravg - pavg) / (pavg * launches_per_interval), 5)}


def time_steps(sim, n):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    sim.step(n)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def secondary_fp64(w, steps):
    """FP64 throughput in the tuned tile of the grid, with the roofline of
    its dominant kernel (launch-by-launch HIP events on the handle's
    stream)."""
    from paper_2401_07416_amd import tdse, tuning
    sim = tdse.sim_from_workload(w, precision="f64", steps=steps + 20)
    t = tuning.tile_for(w, "f64")
    if t:
        sim.set_tile(**t)
    sim.step(20)
    sim.timing_read_split()
    sim.set_timing(True)
    ms = time_steps(sim, steps)
    sim.set_timing(False)
    kt = sim.timing_read_split()
    v = w.cells * steps / (ms * 1e-3) / 1e9
    tile = sim.get_tile().as_dict()
    out = {"workload": w.name + " FP64", "value": round(v, 2), "unit": "Gcell-steps/s",
           "ms_per_step": round(ms / steps, 4), "steps": steps, "tile": tile,
           "roofline": roofline_of(kt, w.cells, "f64", w.name, tile)}
    del sim
    import torch
    torch.cuda.empty_cache()
    return out


def secondary_free_gaussian(reps=5):
    """The 64^3 free packet in FP64 (atomic units, 200 steps at half the
    bound) in full, on the tuned tile of the grid: 2 MB per array, so it
    runs from the caches and says nothing about HBM."""
    from paper_2401_07416_amd import tdse, tuning, workloads
    w = workloads.c1_free_gaussian()
    sim = tdse.sim_from_workload(w, precision="f64", steps=(reps + 1) * w.steps)
    t = tuning.tile_for(w, "f64")
    if t:
        sim.set_tile(**t)
    sim.step(w.steps)
    ms = min(time_steps(sim, w.steps) for _ in range(reps))
    return {"workload": w.name, "value": round(w.cells * w.steps / (ms * 1e-3) / 1e9, 2),
            "unit": "Gcell-steps/s", "ms_per_run": round(ms, 3), "steps": w.steps,
            "tile": sim.get_tile().as_dict(), "cache_resident": True,
            "note": "best of %d runs of the whole 200-step workload" % reps}


def secondary_interp():
    """Unit-cell interpolation (section 2.3) onto the 512x512x1024 FP32 mesh
    from a 24x28x360-sample cell table: the paper's pipeline bottleneck
    (step (ii) of section 3.2), here one HBM-bound setup kernel."""
    import torch

    from paper_2401_07416_amd import tdse, workloads
    table = torch.from_numpy(workloads.unit_cell_table()).cuda()
    d = tdse.make_desc(512, 512, 1024, 0.2, 0.2, 0.2, 0.6582119569, 0.0568563, precision="f32")
    s = tdse.Sim(d, pingpong=False)
    sp = (2.556 / 24, 4.427 / 28, 0.2)
    s.interpolate_potential(table, sp)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record(s.stream)
    for _ in range(reps):
        s.interpolate_potential(table, sp)
    e1.record(s.stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    cells = 512 * 512 * 1024
    wgbs = 4 * cells / (ms * 1e-3) / 1e9
    # the practical ceiling of a write-only kernel on this device (1 GiB
    # fill with 16-byte non-temporal stores), measured in the same process
    fill = tdse.hbm_probe("fill", gib=1.0, reps=16)
    return {"workload": "unit-cell table 24x28x360 -> 512x512x1024 FP32 mesh", "ms": round(ms, 3),
            "gcells_per_s": round(cells / (ms * 1e-3) / 1e9, 1), "write_gbs": round(wgbs, 1),
            "frac_of_peak": round(wgbs / 8000.0, 4), "write_probe_gbs": round(fill, 1),
            "frac_of_write_probe": round(wgbs / fill, 3)}


def secondary_dissim(K=879, T=77, P=128 * 128):
    """Eq. (16) over the paper's sample size (879 trajectories), 77 frames
    of 128x128 detector pixels, FP32 frames: the Gram contraction on the FP64
    matrix cores (2 flops per pair, frame and pixel, against the 78.6 TFLOP/s
    dense FP64 matrix peak)."""
    import torch

    from paper_2401_07416_amd import tdse
    g = torch.Generator(device="cuda")
    g.manual_seed(16)
    frames = torch.rand((K, T, P), generator=g, device="cuda", dtype=torch.float32)
    w = torch.full((T,), 1.0 / T, dtype=torch.float64, device="cuda")
    tdse.dissimilarity(frames, w, 0.04)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record()
    for _ in range(reps):
        tdse.dissimilarity(frames, w, 0.04)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    pp = K * (K - 1) / 2 * T * P
    tf = 2.0 * pp / (ms * 1e-3) / 1e12
    return {"workload": f"d_kj of {K} trajectories x {T} frames x {P} pixels, FP32", "ms": round(ms, 2),
            "g_pair_pixels_s": round(pp / (ms * 1e-3) / 1e9, 1), "tflops_alg": round(tf, 1),
            "bound": "mfma", "peak_tflops_fp64_matrix": 78.6, "frac": round(tf / 78.6, 4)}


def secondary_paper(steps=400):
    """The paper's own Cu(111) set-up (240x240x420 grid plus 100 appended CAP
    planes, interpolated cell potential, eq. (10) CAP, eq. (11) time step,
    h = 20), FP32: the workload of the paper's per-step timings."""
    from paper_2401_07416_amd import tdse, tuning, workloads
    w = workloads.paper_cu111()
    sim = tdse.sim_from_workload(w, precision="f32", steps=steps + 20)
    t = tuning.tile_for(w, "f32")
    if t:
        sim.set_tile(**t)
    sim.step(20)
    ms = time_steps(sim, steps)
    v = w.cells * steps / (ms * 1e-3) / 1e9
    k620_s_per_step = 0.16
    out = {"workload": w.name + " FP32", "value": round(v, 2), "unit": "Gcell-steps/s",
           "ms_per_step": round(ms / steps, 4), "steps": steps,
           "paper_k620_s_per_step": k620_s_per_step,
           "speedup_over_paper_gpu": round(k620_s_per_step / (ms / steps * 1e-3), 1)}
    out["paper_design"] = paper_design(sim, w, v)
    return out


def paper_design(sim, w, ours, steps=100):
    """The section 2.2 design on this device (z-fastest arrays, eq. (12)
    blocks, one launch per half-step, no LDS), for the block shapes of the
    paper's Table 1: Gcell-steps/s and the HBM rate at its algorithmic 32 B
    per FP32 cell-step (each half-step reads S, V, U and writes U)."""
    import torch
    R = sim.psi_r.permute(2, 1, 0).contiguous()
    I = sim.psi_i.permute(2, 1, 0).contiguous()
    V = sim.v.permute(2, 1, 0).contiguous()
    res = {}
    for block in ((16, 4, 2), (16, 4, 4), (16, 8, 4), (16, 8, 8), (64, 4, 1), (64, 1, 4)):
        sim.paper_layout_run(R, I, V, 10, block)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        sim.paper_layout_run(R, I, V, steps, block)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        g = w.cells * steps / (ms * 1e-3) / 1e9
        res["x".join(map(str, block))] = {"gcell_steps_s": round(g, 2),
                                          "ms_per_step": round(ms / steps, 4),
                                          "hbm_gbs_alg": round(g * 32, 1)}
    best = max(res, key=lambda k: res[k]["gcell_steps_s"])
    return {"blocks": res, "best_block": best,
            "library_over_paper_design": round(ours / res[best]["gcell_steps_s"], 2),
            "library_over_paper_block_16x4x4": round(ours / res["16x4x4"]["gcell_steps_s"], 2)}


def secondary_shard(steps=400):
    """One GPU's z-slab of the headline grid split over 8 GPUs (512x512x128,
    periodic z in place of the halo planes), with the halo traffic the
    sharded sweep would exchange per two-step pass: R^n on 4 planes below
    and 3 above the slab, I^{n-1/2} on 3 below and 2 above (the planes the
    sweep's first and last stored planes depend on), over one xGMI link to
    each z neighbour at the 153 GB/s per link of the MI355X's
    specification (an estimate; nothing here uses a second GPU)."""
    from paper_2401_07416_amd import tdse, tuning, workloads
    w = workloads.c3_shard(8, 1)
    sim = tdse.sim_from_workload(w, precision="f32", steps=steps + 20)
    t = tuning.tile_for(w, "f32")
    if t:
        sim.set_tile(**t)
    sim.step(20)
    ms = time_steps(sim, steps)
    v = w.cells * steps / (ms * 1e-3) / 1e9
    plane = w.nx * w.ny * 4
    up, down = (3 + 2) * plane, (4 + 3) * plane
    link_us = max(up, down) / 153e9 * 1e6
    pass_us = 2 * ms / steps * 1e3
    tile = sim.get_tile()
    return {"workload": w.name + " FP32 (one of 8 z-slabs of surface-512x512x1024)",
            "value": round(v, 2), "unit": "Gcell-steps/s", "ms_per_step": round(ms / steps, 4),
            "two_step": int(tile.two_step), "halo_bytes_per_pass": up + down,
            "halo_link_us_per_pass_est": round(link_us, 1), "compute_us_per_pass": round(pass_us, 1),
            "eight_gpu_gcell_steps_s_if_hidden": round(8 * v, 1)}


def secondary_adjoint():
    """Plain forward, checkpointed forward and adjoint of the 128x128x256,
    4000-step gradient workload in FP32, timed with HIP events."""
    import torch

    from paper_2401_07416_amd import autograd as tag
    from paper_2401_07416_amd import workloads
    w = workloads.c5_adjoint()
    prob = tag.problem_for(w, precision="f32", ckpt_every=100)

    def fresh():
        s = prob.make_sim()
        s.build_potential(w.atoms, soft=w.soft, cutoff=w.cutoff, kappa=w.kappa, a0=w.a0)
        s.set_cap_quadratic(*w.cap)
        s.finalize()
        s.init_gaussian(w.r0, prob.k0(), w.sigma)
        return s

    warm = fresh()
    time_steps(warm, 200)
    del warm
    ms_plain = time_steps(fresh(), w.steps)
    sim = fresh()
    sim.bind_adjoint(w.steps, 100)
    ms_fwd = time_steps(sim, w.steps)
    rb = torch.full((w.n_records(), w.ny, w.nx), 1e-3, dtype=torch.float32, device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    gV, _, _ = sim.adjoint(rb)
    e1.record()
    torch.cuda.synchronize()
    ms_adj = e0.elapsed_time(e1)
    cs = w.cells * w.steps
    return {"workload": w.name + " FP32, 4000 steps, checkpoints every 100",
            "plain_forward_ms": round(ms_plain, 2),
            "checkpointed_forward_ms": round(ms_fwd, 2), "adjoint_ms": round(ms_adj, 2),
            "adjoint_over_plain": round((ms_fwd + ms_adj) / ms_plain, 2),
            "plain_gcell_steps_s": round(cs / (ms_plain * 1e-3) / 1e9, 1),
            "backward_gcell_steps_s": round(cs / (ms_adj * 1e-3) / 1e9, 1),
            "grad_finite": bool(torch.isfinite(gV).all())}


def secondary_batch(n_configs=64, batch_steps=1000, single_steps=100):
    """The 64 uneven film grids stepped as one batch (one launch per step,
    a graph per 50-step record interval) against the same grids run one at
    a time with the plain path, FP32."""
    import torch

    from paper_2401_07416_amd import tdse, workloads
    ws = workloads.c4_batch(n_configs, steps=batch_steps + single_steps + 100)
    b = tdse.batch_from_workloads(ws, precision="f32", steps=batch_steps + single_steps + 100)
    b.prepare()
    b.run(50)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.run(batch_steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1)
    cells = sum(w.cells for w in ws)
    ok = all(st == tdse.OK for st in b.status())
    ms_s = 0.0
    with torch.cuda.stream(b.stream):
        for m in b.members:
            a0 = torch.cuda.Event(enable_timing=True)
            a1 = torch.cuda.Event(enable_timing=True)
            a0.record(b.stream)
            m.step(single_steps)
            a1.record(b.stream)
            a1.synchronize()
            ms_s += a0.elapsed_time(a1)
    vb = cells * batch_steps / (ms_b * 1e-3) / 1e9
    vs = cells * single_steps / (ms_s * 1e-3) / 1e9
    b.close()
    return {"workload": f"{n_configs} film grids 128^2x256..256^2x512, {cells} cells, FP32",
            "batched_gcell_steps_s": round(vb, 1), "one_at_a_time_gcell_steps_s": round(vs, 1),
            "batched_over_plain": round(vb / vs, 3), "status_ok": ok,
            "note": "working set 21 GB >> 256 MB MALL"}


def copy_probe():
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                      "launches": 5}), flush=True)


def _sec_fp64_c2():
    from paper_2401_07416_amd import workloads
    return secondary_fp64(workloads.c2_surface(), 400)


def _sec_fp64_c3():
    from paper_2401_07416_amd import workloads
    return secondary_fp64(workloads.c3_headline(), 100)


# the secondary measurements of the bench line, in the order they run
SECONDARIES = {"fp64": _sec_fp64_c2, "fp64_headline_grid": _sec_fp64_c3,
               "free_gaussian_64cubed": secondary_free_gaussian, "adjoint": secondary_adjoint,
               "batched": secondary_batch, "interpolation": secondary_interp,
               "dissimilarity": secondary_dissim, "paper_setup": secondary_paper,
               "shard_share": secondary_shard}


def main():
    a = parse()
    if a.cpu_child:
        cpu_child(a)
        return
    if a.copy_probe:
        copy_probe()
        return
    if a.only:
        print(json.dumps({a.only: SECONDARIES[a.only]()}), flush=True)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "libtdse runs on one GPU; a sharded multi-GPU path is not "
                                   "implemented, so only --gpus 1 is measured",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import torch

    from paper_2401_07416_amd import tdse, tuning, workloads
    w = workloads.ALL[a.workload]()
    prec = a.precision
    total = a.warmup + a.steps
    # capacity for the record-cost window after the timed region
    rec_window = 4 * w.record_every if w.record_every else 0
    sim = tdse.sim_from_workload(w, precision=prec, steps=total + rec_window)
    tile = json.loads(a.tile) if a.tile else tuning.tile_for(w, prec)
    if tile is not None:
        sim.set_tile(**tile)
    t = sim.get_tile()
    torch.cuda.synchronize()
    # The practical ceiling: streaming kernels with the copy's and the
    # step's mix of read and written streams, 1 GiB per stream.  Measured
    # before the warm-up steps: its ~25 ms of streaming also carries the
    # device through the clock transient that follows the compute-bound
    # potential build (without it, the sweep's launches 2-15 after the build
    # run up to 17% slower than the steady state).
    practical = None
    if not a.no_timing:
        try:
            copy_gbs = tdse.hbm_probe("copy", reps=16)
            mix_gbs = tdse.hbm_probe("mix", reps=16)
            practical = {"copy_gbs": round(copy_gbs, 1), "mix_gbs": round(mix_gbs, 1)}
        except Exception as e:  # measurement context only
            practical = {"error": str(e)}
        torch.cuda.empty_cache()
    # The records (eq. (15), every h steps) cost, on a window of whole record
    # intervals.  Measured before the warm-up steps: the sweep's launches
    # after the set-up run up to 10% slower than the steady state for about
    # 20 ms (a device transient the probe above does not remove), which a
    # short timed window would otherwise mostly consist of.
    rec_cost = None
    if not a.no_timing and rec_window:
        try:
            rec_cost = record_cost(sim, w)
            if rec_cost is not None:
                rec_cost["measured"] = "before the warm-up steps"
        except Exception as e:  # measurement context only
            rec_cost = {"error": repr(e)}
    sim.step(a.warmup)
    torch.cuda.synchronize()
    sim.timing_read_split()
    sim.set_timing(not a.no_timing)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record()
    sim.step(a.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = e0.elapsed_time(e1)
    sim.set_timing(False)
    kt = sim.timing_read_split()
    det = sim.detect()
    cells = w.cells
    value = cells * a.steps / (ms * 1e-3) / 1e9
    roof = None if a.no_timing else roofline_of(kt, cells, prec, w.name, t.as_dict())
    # algorithmic bytes per cell-step of the launches the timed steps ran
    es = 8 if prec == "f64" else 4
    alg_words = sum(WORDS[k.replace("_rec", "")] * v[1] for k, v in kt.items())
    bytes_per_cell_step = es * alg_words / max(1, a.steps)
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gcell-steps/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(ms / a.steps, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec,
        "data": "synthetic",
        "config": {"workload": f"{w.name} (FP32 state, FP64 sums)" if prec == "f32" else w.name,
                   "grid": [w.nx, w.ny, w.nz], "cells": cells, "record_every": w.record_every,
                   "k_det": w.k_det, "cap_planes": list(w.cap[:2]) if w.cap else None,
                   "atoms": int(len(w.atoms)) if w.atoms is not None else 0,
                   "tile": t.as_dict(),
                   "dt": det.dt, "records": det.n_records},
        "roofline": roof,
        "wall_s": round(wall, 3),
        "hbm_bytes_per_cell_step_alg": bytes_per_cell_step,
        "hbm_gbs_whole_step": round(value * bytes_per_cell_step, 1),
    }
    if rec_cost is not None:
        out["record_cost"] = rec_cost
    del sim
    torch.cuda.empty_cache()
    if roof is not None and practical is not None:
        if "mix_gbs" in practical:
            practical["frac_of_mix"] = round(roof["achieved"] / practical["mix_gbs"], 4)
        roof["practical"] = practical
    fp64_c2 = None
    if not a.no_secondary:
        sec = {}
        for name, fn in SECONDARIES.items():
            try:
                sec[name] = fn()
            except Exception as ex:  # reported, never hidden
                sec[name] = {"error": repr(ex)}
            torch.cuda.empty_cache()
        out["secondary"] = sec
        fp64_c2 = sec["fp64"].get("value")
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a, value, fp64_c2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

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
per cell in FP32 (read R, I, V once, write R, I once: two steps for the
sweep, one for the one-pass step; 16 B for a half-step), divided by its
average launch time measured with HIP events around each launch inside the
timed region, on the stream the kernels run on.  traffic: calibrated
rocprofv3 FETCH_SIZE + WRITE_SIZE per launch from profiles/, while the
kernel sources and tile match.  cpu_baseline: the FP64 oracle timed on this
host's cores on a bounded slab of the same workload.
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
    p.add_argument("--cpu-seconds", type=float, default=15.0,
                   help="target CPU time of the timed oracle sample")
    p.add_argument("--cpu-planes", type=int, default=48)
    p.add_argument("--no-timing", action="store_true",
                   help="do not bracket launches with events (value only)")
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


def cpu_baseline(w, seconds, planes):
    """Time the FP64 oracle on a slab of `planes` z-planes of the workload
    (the windowed potential and packet of the full grid, zero outside the
    slab) for about `seconds` of wall time, on the host threads the oracle
    is given (at most 16, the CPU share of one GPU)."""
    import numpy as np

    import oracle
    threads = min(16, len(os.sched_getaffinity(0)))
    oracle.set_threads(threads)
    g = oracle.Grid(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.hbar, w.mass, bc=w.bc)
    k0c = int(round(w.r0[2] / w.dz)) - planes // 2
    size = (w.nx, w.ny, planes)
    V = oracle.potential_window(g, w.atoms, (0, 0, k0c), size, soft=w.soft, cutoff=w.cutoff,
                                kappa=w.kappa, a0=w.a0, screened=w.screened)
    # time step of the full grid: the slab holds the deepest wells
    Vs = oracle.potential_window(g, w.atoms, (0, 0, int(30.5 / w.dz) - 8), (w.nx, w.ny, 40),
                                 soft=w.soft, cutoff=w.cutoff, kappa=w.kappa, a0=w.a0,
                                 screened=w.screened)
    gs = oracle.Grid(w.nx, w.ny, 40, w.dx, w.dy, w.dz, w.hbar, w.mass)
    dt = w.dt_frac * w.hbar / oracle.emax(gs, Vs)
    k0 = oracle.wavevector(w.energy, w.hbar, w.mass) * np.array(w.k_dir)
    R, I = oracle.init_gaussian_window(g, w.r0, k0, w.sigma, dt, (0, 0, k0c), size)
    gw = oracle.Grid(w.nx, w.ny, planes, w.dx, w.dy, w.dz, w.hbar, w.mass, bc=(0, 0, 1))
    s = oracle.Sim(gw, V, R, I, dt, k_det=planes // 2)
    t0 = time.perf_counter()
    s.step(2)
    per = (time.perf_counter() - t0) / 2
    steps = max(2, int(seconds / per))
    t0 = time.perf_counter()
    s.step(steps)
    el = time.perf_counter() - t0
    threads = oracle.get_threads()
    cells = w.nx * w.ny * planes
    out = {"value": cells * steps / el / 1e9, "unit": "Gcell-steps/s", "cores": threads,
           "kind": "oracle",
           "sample": f"FP64 oracle, {w.nx}x{w.ny}x{planes}-plane slab of the {w.name} grid "
                     f"around the packet, {steps} steps, {el:.1f} s",
           "ns_per_cell_step": el / (cells * steps) * 1e9}
    # the serial analogue (one core), on the same slab for about a quarter of
    # the time
    oracle.set_threads(1)
    t0 = time.perf_counter()
    s.step(1)
    per1 = time.perf_counter() - t0
    steps1 = max(1, int(seconds / 4 / per1))
    t0 = time.perf_counter()
    s.step(steps1)
    el1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    out["single_core"] = {"value": cells * steps1 / el1 / 1e9, "cores": 1, "steps": steps1,
                          "ns_per_cell_step": el1 / (cells * steps1) * 1e9}
    return out


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


def secondary_fp64(steps=400):
    """FP64 throughput on the 256x256x512 surface grid (one-pass step)."""
    from paper_2401_07416_amd import tdse, tuning, workloads
    w = workloads.c2_surface()
    sim = tdse.sim_from_workload(w, precision="f64", steps=steps + 20)
    t = tuning.tile_for(w, "f64")
    if t:
        sim.set_tile(**t)
    sim.step(20)
    ms = time_steps(sim, steps)
    v = w.cells * steps / (ms * 1e-3) / 1e9
    return {"workload": w.name + " FP64", "value": round(v, 2), "unit": "Gcell-steps/s",
            "ms_per_step": round(ms / steps, 4),
            "hbm_gbs_alg": round(v * 40, 1), "steps": steps}


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
    return {"workload": "unit-cell table 24x28x360 -> 512x512x1024 FP32 mesh", "ms": round(ms, 3),
            "gcells_per_s": round(cells / (ms * 1e-3) / 1e9, 1),
            "write_gbs": round(4 * cells / (ms * 1e-3) / 1e9, 1)}


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


def secondary_batch(n_configs=64, batch_steps=400, single_steps=100):
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


def main():
    a = parse()
    if a.copy_probe:
        copy_probe()
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
    sim = tdse.sim_from_workload(w, precision=prec, steps=total)
    tile = json.loads(a.tile) if a.tile else tuning.tile_for(w, prec)
    if tile is not None:
        sim.set_tile(**tile)
    t = sim.get_tile()
    torch.cuda.synchronize()
    sim.step(a.warmup)
    torch.cuda.synchronize()
    sim.timing_read()
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
    kt = sim.timing_read()
    det = sim.detect()
    cells = w.cells
    value = cells * a.steps / (ms * 1e-3) / 1e9
    es = 8 if prec == "f64" else 4
    # algorithmic bytes per launch: a half-step reads the stencil array, the
    # updated array and V and writes the updated array (4 words per cell); the
    # one-pass step reads R, I, V and writes R, I (5 words per cell); the
    # two-step sweep moves the same 5 words per cell for two steps
    words = {"half_i": 4, "half_r": 4, "fused": 5, "two_step": 5}
    names = {"half_i": "half_step eq.(9) imaginary", "half_r": "half_step eq.(8) real",
             "fused": "fused_step eqs.(9)+(8) one-pass",
             "two_step": "fused2 two-step sweep eqs.(9)+(8)+(9)+(8)"}
    roof = None
    dom = max(kt, key=lambda k: kt[k][0])
    tot_ms, launches = kt[dom]
    if launches:
        avg = tot_ms / launches
        alg_bytes = words[dom] * es * cells
        achieved = alg_bytes / (avg * 1e-3) / 1e9
        traffic = traffic_from_profiles(w.name, prec, dom, t.as_dict())
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "frac_at_32B_per_cell_step": round(value * 32 / HBM_PEAK_GBS, 4),
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "kernel": names[dom], "avg_launch_ms": round(avg, 5),
                "alg_bytes_per_launch": alg_bytes,
                "launches": {k: v[1] for k, v in kt.items()},
                "kernel_ms": {k: round(v[0], 3) for k, v in kt.items()}}
        if traffic is not None:
            # the memory-side rate: counted bytes per launch over this run's
            # average launch time
            roof["traffic_gbs"] = round(traffic / (avg * 1e-3) / 1e9, 1)
            roof["traffic_frac"] = round(traffic / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    # algorithmic bytes per cell-step of the launches the timed steps ran
    alg_words = sum(words[k] * kt[k][1] for k in kt)
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
    if roof is not None:
        # the practical ceiling: streaming kernels with the copy's and the
        # one-pass step's mix of read and written streams, 1 GiB per stream
        try:
            copy_gbs = tdse.hbm_probe("copy")
            mix_gbs = tdse.hbm_probe("mix")
            roof["practical"] = {"copy_gbs": round(copy_gbs, 1), "mix_gbs": round(mix_gbs, 1),
                                 "frac_of_mix": round(roof["achieved"] / mix_gbs, 4)}
        except Exception as e:  # measurement context only
            roof["practical"] = {"error": str(e)}
        torch.cuda.empty_cache()
    if not a.no_secondary:
        sec = {}
        for name, fn in (("fp64", secondary_fp64), ("adjoint", secondary_adjoint),
                         ("batched", secondary_batch), ("interpolation", secondary_interp),
                         ("dissimilarity", secondary_dissim), ("paper_setup", secondary_paper),
                         ("shard_share", secondary_shard)):
            try:
                sec[name] = fn()
            except Exception as ex:  # reported, never hidden
                sec[name] = {"error": repr(ex)}
        out["secondary"] = sec
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds, a.cpu_planes)
        out["cpu_baseline"]["speedup_gpu_over_cpu"] = round(value / out["cpu_baseline"]["value"], 1)
        sc = out["cpu_baseline"]["single_core"]
        sc["speedup_gpu_over_single_core"] = round(value / sc["value"], 1)
        sc["paper_speedup_over_serial_cpu"] = 350
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

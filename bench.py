#!/usr/bin/env python3
"""Throughput of the LBM time step on one MI355X.

Default workload: D3Q19, 256^3 fully periodic, FP64, 3D Taylor-Green vortex
(U0 = 0.05) plus U(-1e-6, 1e-6) population noise (seed 2), tau = 0.6.  A
timed step is one lbm_step(1) -- pull-stream, bounce-back, moments,
equilibrium, IMEX-BGK relaxation, forcing and store fused in one kernel --
and the timed region ends with one Monitor reduction (lbm_reduce), as the
paper's main loop monitors every interv steps.

Prints one JSON line: MLUPS (lattice points x steps / time / 1e6, counting
every node of the domain), the HBM roofline of the dominant kernel from
algorithmic bytes per lattice update (2 Q sizeof(storage)) and its average
launch duration measured with HIP events on the launch stream, and the CPU
oracle's MLUPS on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
METRIC = "MLUPS & % of HBM peak, D3Q19 256³ FP64 vs FP16-store; adjoint/forward ratio"
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2, "e4m11": 2}
DTYPE_NAME = {"f64": "f64", "f32": "f32", "f16": "f16-store/f32", "bf16": "bf16-store/f32",
              "e4m11": "e4m11-store/f32"}


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    # 100 untimed steps: after the host-side input generation leaves the GPU
    # idle, the short FP16 launches take ~100 launches (~20 ms) to reach
    # their steady duration (FP64: ~5).
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=256, help="cube edge of the workload")
    ap.add_argument("--storage", default="f64", choices=sorted(STORAGE_BYTES))
    ap.add_argument("--pattern", default="ab", choices=["ab", "aa"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the extra lines (FP16 storage, compressible model, the other "
                         "pattern, 2000-step run, precision, adjoint, channels, sphere box, D2Q9 "
                         "boxes)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of the population buffer size "
                         "(reference point for HBM byte counters)")
    ap.add_argument("--only", choices=sorted(EXTRA_LINES),
                    help="run just this extra line (no main line, no CPU baseline) and print "
                         "its JSON object")
    return ap.parse_args()


def run_gpu(n, storage, pattern, steps, warmup, copy_probe=False, compressible=False):
    import numpy as np
    import torch

    from paper_2201_11330_amd import lbm
    from paper_2201_11330_amd import workloads as W

    dims = (n, n, n)
    rho, u = W.taylor_green_3d(n, U0=0.05)
    noise = W.population_noise(W.D3Q19, dims, 1e-6, seed=2)
    torch.cuda.set_device(0)
    sim = lbm.LBM(lbm.D3Q19, n, n, n, 0.6, storage=storage, aa=(pattern == "aa"),
                  compressible=compressible)
    sim.init_equilibrium(rho, u, noise)
    del noise
    stream = sim.stream
    red0 = sim.reduce()
    for _ in range(warmup):
        sim.step(1)
    torch.cuda.synchronize()

    # One event pair around the K launches (their average duration, launch
    # gaps included) and one more after the closing Monitor reduction.
    e_start, e_steps, e_end = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    with torch.cuda.stream(stream):
        e_start.record(stream)
        for _ in range(steps):
            sim.step(1)
        e_steps.record(stream)
        red = sim.reduce()  # Monitor: synchronises the stream
        e_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    launch_ms = e_start.elapsed_time(e_steps) / steps
    total_ms = e_start.elapsed_time(e_end)
    result = {
        "dims": dims,
        "storage": storage,
        "pattern": pattern,
        "total_ms": total_ms,
        "wall_s": wall,
        "launch_ms_mean": launch_ms,
        "mass_drift": abs(red["mass"] - red0["mass"]) / red0["mass"],
        "ke_ratio": red["ke"] / red0["ke"],
        "unstable": red["unstable"],
    }
    sim.close()
    if copy_probe:
        nbytes = 19 * n ** 3 * STORAGE_BYTES[storage]
        a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        reps = 20
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        result["copy_probe"] = {"bytes": nbytes, "ms": ms, "gbs": 2 * nbytes / ms / 1e6}
    return result


def run_channel(steps=200, warmup=10, nx=512, ny=128, nz=128, tau=0.9, g=1e-6, nodal=False):
    """Forced channel 512 x 128 x 128 (x, z periodic; solid planes y = 0 and
    ny-1 with halfway bounce-back, or with nodal=True wall nodes of the
    modified nodal scheme on those planes; g_x = 1e-6; start rho = 1,
    u ~ U(+-1e-4), seed 3): the paper's benchmark box shape.  MLUPS counts
    every node of the domain (the paper's definition) and, separately,
    fluid nodes."""
    import torch

    from paper_2201_11330_amd import lbm
    from paper_2201_11330_amd import workloads as W

    bc = (W.PERIODIC, W.WALLS_NODAL if nodal else W.SOLID_ENDS, W.PERIODIC)
    rho, u = W.channel(nx, ny, nz, amplitude=1e-4, seed=3, bc=(W.PERIODIC, W.SOLID_ENDS, W.PERIODIC))
    if nodal:  # wall nodes at rest
        u[:, :, [0, ny - 1], :] = 0.0
    sim = lbm.LBM(lbm.D3Q19, nx, ny, nz, tau, force=(g, 0.0, 0.0), bc=bc)
    sim.init_equilibrium(rho, u)
    sim.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sim.close()
    nodes = nx * ny * nz
    mlups = nodes * steps / (ms * 1e-3) / 1e6
    fluid = ny if nodal else ny - 2
    walls = "nodal wall nodes" if nodal else "solid planes"
    return {"workload": f"D3Q19 {nx}x{ny}x{nz} channel, {walls} y=0,{ny - 1}, g_x={g}, tau={tau}, "
                        f"FP64 AB, {steps} steps",
            "mlups": round(mlups, 1), "mlups_fluid_nodes": round(mlups * fluid / ny, 1),
            "achieved_gbs": round(304 * nodes * steps / (ms * 1e-3) / 1e9, 1)}


def run_channel_sustained(steps=20000, chunk=1000, warmup=10, nx=512, ny=128, nz=128, tau=0.9,
                          g=1e-6):
    """The channel workload at its stated length: 20,000 steps of the
    512 x 128 x 128 box (halfway walls, g_x = 1e-6, tau = 0.9), issued as
    lbm_step(chunk) calls with an event on the launch stream after each, so
    that the throughput of every chunk shows how it changes over the run."""
    import torch

    from paper_2201_11330_amd import lbm
    from paper_2201_11330_amd import workloads as W

    bc = (W.PERIODIC, W.SOLID_ENDS, W.PERIODIC)
    rho, u = W.channel(nx, ny, nz, amplitude=1e-4, seed=3, bc=bc)
    sim = lbm.LBM(lbm.D3Q19, nx, ny, nz, tau, force=(g, 0.0, 0.0), bc=bc)
    sim.init_equilibrium(rho, u)
    del rho, u
    sim.step(warmup)
    torch.cuda.synchronize()
    nchunks = steps // chunk
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nchunks + 1)]
    wall0 = time.perf_counter()
    ev[0].record(sim.stream)
    for i in range(nchunks):
        sim.step(chunk)
        ev[i + 1].record(sim.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    sim.close()
    nodes = nx * ny * nz
    ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(nchunks)]
    per = [nodes * chunk / (m * 1e-3) / 1e6 for m in ms]
    total = sum(ms)
    mlups = nodes * chunk * nchunks / (total * 1e-3) / 1e6
    return {"workload": f"D3Q19 {nx}x{ny}x{nz} channel, solid planes y=0,{ny - 1}, g_x={g}, "
                        f"tau={tau}, FP64 AB, {chunk * nchunks} steps ({nchunks} x lbm_step({chunk}))",
            "mlups": round(mlups, 1),
            "achieved_gbs": round(304 * nodes * chunk * nchunks / (total * 1e-3) / 1e9, 1),
            "frac": round(304 * nodes * chunk * nchunks / (total * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "us_per_step": round(total * 1e3 / (chunk * nchunks), 2),
            "chunk_mlups_first_last": [round(per[0], 1), round(per[-1], 1)],
            "chunk_mlups_min_max": [round(min(per), 1), round(max(per), 1)],
            "wall_s": round(wall, 3)}


def run_taylor_green_sustained(n=256, steps=2000, chunk=250, warmup=100, tau=0.6):
    """The headline workload (D3Q19 n^3 periodic FP64 Taylor-Green with
    1e-6 noise, seed 2) for `steps` steps issued as lbm_step(chunk) calls,
    an event on the launch stream after each: the sustained rate of the
    benchmark's step kernel and how it changes over the run."""
    import torch

    from paper_2201_11330_amd import lbm
    from paper_2201_11330_amd import workloads as W

    rho, u = W.taylor_green_3d(n, U0=0.05)
    noise = W.population_noise(W.D3Q19, (n, n, n), 1e-6, seed=2)
    sim = lbm.LBM(lbm.D3Q19, n, n, n, tau)
    sim.init_equilibrium(rho, u, noise)
    del rho, u, noise
    sim.step(warmup)
    torch.cuda.synchronize()
    nchunks = steps // chunk
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nchunks + 1)]
    wall0 = time.perf_counter()
    ev[0].record(sim.stream)
    for i in range(nchunks):
        sim.step(chunk)
        ev[i + 1].record(sim.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    sim.close()
    nodes = n ** 3
    ms = [ev[i].elapsed_time(ev[i + 1]) for i in range(nchunks)]
    per = [nodes * chunk / (m * 1e-3) / 1e6 for m in ms]
    total = sum(ms)
    gbs = 304 * nodes * chunk * nchunks / (total * 1e-3) / 1e9
    return {"workload": f"D3Q19 {n}^3 periodic FP64 Taylor-Green, tau={tau}, {chunk * nchunks} steps "
                        f"({nchunks} x lbm_step({chunk})) after {warmup} untimed",
            "kernel": step_kernel_name(n, "f64", "ab"),
            "mlups": round(nodes * chunk * nchunks / (total * 1e-3) / 1e6, 1),
            "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "us_per_step": round(total * 1e3 / (chunk * nchunks), 2),
            "chunk_mlups_first_last": [round(per[0], 1), round(per[-1], 1)],
            "chunk_mlups_min_max": [round(min(per), 1), round(max(per), 1)],
            "wall_s": round(wall, 3)}


def _tg_decay(n, storage, steps, every, rho, u, noise, tau=0.6):
    """One Taylor-Green run sampled every `every` steps: kinetic energies,
    summed step time (an event pair around each lbm_step(every)) and the
    final velocity."""
    import torch

    from paper_2201_11330_amd import lbm

    sim = lbm.LBM(lbm.D3Q19, n, n, n, tau, storage=storage)
    sim.init_equilibrium(rho, u, noise)
    ts, ke, ms = [], [], 0.0
    for it in range(0, steps + 1, every):
        ts.append(it)
        ke.append(sim.reduce()["ke"])
        if it < steps:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(sim.stream)
            sim.step(every)
            e1.record(sim.stream)
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
    _, uN = sim.moments(dtype=torch.float32 if storage != "f64" else torch.float64)
    sim.close()
    return ts, ke, ms, uN


def ke_decay_rate(ts, ke, skip=100):
    """Least-squares slope of -ln KE(t) over the samples with t >= skip (the
    first steps carry the start-up transient of the equilibrium start)."""
    import numpy as np

    ts, ke = np.asarray(ts, float), np.asarray(ke, float)
    m = ts >= skip
    return float(-np.polyfit(ts[m], np.log(ke[m]), 1)[0])


def run_precision(n=512, steps=500, every=10, U0=0.05, tau=0.6):
    """Reduced-precision workload: D3Q19 n^3 Taylor-Green, tau = 0.6, 500
    steps, populations stored as f - w in FP16 and BF16 (and FP32) with FP32
    arithmetic, each against the FP64 run on the same inputs (population
    noise U(+-1e-6) from torch's seeded device generator, seed 4): MLUPS of
    the steps, max |u - u_f64| and the relative error of the kinetic-energy
    decay rate (KE sampled every 10 steps, fitted from step 100)."""
    import torch

    from paper_2201_11330_amd import workloads as W

    rho, u = W.taylor_green_3d(n, U0=U0)
    rho = torch.from_numpy(rho).cuda()
    u = torch.from_numpy(u).cuda()
    noise = W.uniform_noise_device((19, n, n, n), 1e-6, seed=4)
    nodes = n ** 3
    out = {"workload": f"D3Q19 {n}^3 periodic 3D Taylor-Green U0={U0} + 1e-6 noise (device "
                       f"generator, seed 4), tau={tau}, {steps} steps, KE every {every} steps"}
    ts, ke64, ms64, u64 = _tg_decay(n, "f64", steps, every, rho, u, noise, tau)
    r64 = ke_decay_rate(ts, ke64)
    m64 = nodes * steps / (ms64 * 1e-3) / 1e6
    out["f64"] = {"mlups": round(m64, 1), "ke_decay_rate_per_step": r64}
    for storage in ("f16", "e4m11", "bf16", "f32"):
        ts, ke, ms, us = _tg_decay(n, storage, steps, every, rho, u, noise, tau)
        du = (us.to(torch.float64) - u64).abs().max().item()
        del us
        torch.cuda.empty_cache()
        m = nodes * steps / (ms * 1e-3) / 1e6
        blu = 2 * 19 * STORAGE_BYTES[storage]
        out[storage] = {"mlups": round(m, 1), "speedup_vs_f64": round(m / m64, 3),
                        "frac": round(m * blu / 1e3 / HBM_PEAK_GBS, 4),
                        "ke_decay_rate_rel_err": abs(ke_decay_rate(ts, ke) / r64 - 1),
                        "max_abs_du": du, "max_abs_du_over_U0": du / U0}
    return out


def run_paper_sphere(steps=100, warmup=5, storage="f64"):
    """The paper's validation and performance box (Sec. 5-6): D3Q27,
    512 x 128 x 128, solid sphere of radius 8 at (64, 64, 64), 100 steps --
    here in a periodic box driven by g_x = 1e-6 (the paper's inlet, outlet
    and symmetry conditions are not specified).  MLUPS over every lattice
    point of the domain, the paper's definition."""
    import torch

    from paper_2201_11330_amd import lbm
    from paper_2201_11330_amd import workloads as W

    dims = (512, 128, 128)
    nx, ny, nz = dims
    solid = W.sphere_mask(dims, (64, 64, 64), 8)
    rho, u = W.channel(*dims, amplitude=1e-4, seed=7, bc=(0, 0, 0))
    u[:, solid.astype(bool)] = 0.0
    sim = lbm.LBM(lbm.D3Q27, nx, ny, nz, 0.6, force=(1e-6, 0.0, 0.0), storage=storage)
    sim.set_solid(solid)
    sim.init_equilibrium(rho, u)
    sim.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    drag = sim.wall_force()
    sim.close()
    nodes = nx * ny * nz
    blu = 2 * 27 * STORAGE_BYTES[storage] + 4  # + the 4-byte link bits of the mask
    return {"workload": "D3Q27 512x128x128, sphere r=8 at (64,64,64), periodic, g_x=1e-6, "
                        f"tau=0.6, {storage} AB, {steps} steps",
            "mlups": round(nodes * steps / (ms * 1e-3) / 1e6, 1),
            "bytes_per_update": blu,
            "achieved_gbs": round(blu * nodes * steps / (ms * 1e-3) / 1e9, 1),
            "sphere_force_x": drag[0],
            "paper_context": PAPER_CONTEXT}


# The paper's own figures for this box, as context (other hardware, not a
# target).
PAPER_CONTEXT = {
    "hardware": "ThetaGPU node: 2x AMD Rome 64-core CPUs, 8x NVIDIA A100 (Sec. 5, node table)",
    "workload": "flow past a sphere, D3Q27 512x128x128, FP64, inlet/outlet boundaries, 1-8 GPUs",
    "mlups": None,
    "note": "the paper gives its MLUPS in a figure only (Sec. 6), not in its text; its code "
            "profile (Sec. 3: 8 ranks, one A100 each, 6401 steps, 0.11 s in total) samples "
            "host time only. "
            "For scale: an A100's ~1.555 TB/s allows ~3,600 MLUPS at 432 B per D3Q27 FP64 "
            "update (NVIDIA's bandwidth figure, not the paper's)",
}


def run_small_2d(n=128, steps=1000, tau=0.8):
    """D2Q9 n^2 periodic Taylor-Green (U0 = 0.01), the launch-bound small
    workload: MLUPS of lbm_step(steps) (launches of four steps each, LDS
    temporal blocking) issued eagerly and as captured-graph replays."""
    import torch

    from paper_2201_11330_amd import lbm
    from paper_2201_11330_amd import workloads as W

    rho, u = W.taylor_green_2d(n, U0=0.01)
    out = {"workload": f"D2Q9 {n}^2 periodic Taylor-Green, tau={tau}, {steps} steps, FP64 AB",
           "kernel": "k_step_ab_fused2d<16> (4 steps per launch, 16x16-node regions)"}
    for graph in (False, True):
        sim = lbm.LBM(lbm.D2Q9, n, n, 1, tau, graph=graph)
        best = None
        for _ in range(3):
            sim.init_equilibrium(rho, u)
            sim.step(64)  # warm-up (and capture)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(sim.stream)
            sim.step(steps)
            e1.record(sim.stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        sim.close()
        out["mlups_graph" if graph else "mlups"] = round(n * n * steps / (best * 1e-3) / 1e6, 1)
    return out


def run_large_2d(n=4096, steps=200, warmup=400, tau=0.8):
    """D2Q9 n^2 periodic Taylor-Green (U0 = 0.01), FP64 AB: a box far larger
    than the caches, where the four-step launches (strips streamed up the
    rows) read and write the state once per four steps (36 B per update)
    against the 144 B a one-step pass moves.  400 untimed steps: after the
    host-side set-up leaves the GPU idle, these launches take ~50 of them
    (~30 ms) to reach their steady duration (670 -> 487 us)."""
    import torch

    from paper_2201_11330_amd import lbm
    from paper_2201_11330_amd import workloads as W

    rho, u = W.taylor_green_2d(n, U0=0.01)
    sim = lbm.LBM(lbm.D2Q9, n, n, 1, tau)
    sim.init_equilibrium(rho, u)
    del rho, u
    sim.step(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    sim.close()
    mlups = n * n * steps / (ms * 1e-3) / 1e6
    one_step_bound = HBM_PEAK_GBS * 1e3 / 144.0
    return {"workload": f"D2Q9 {n}^2 periodic Taylor-Green, tau={tau}, {steps} steps, FP64 AB",
            "kernel": "k_step_ab_stream2d (4 steps per launch, strips of 224 columns streamed "
                      "up row segments)",
            "mlups": round(mlups, 1), "bytes_per_update_moved": 36,
            "one_step_hbm_bound_mlups": round(one_step_bound, 1),
            "vs_one_step_hbm_bound": round(mlups / one_step_bound, 3)}


def run_adjoint(n=128, steps=500, k=50, storage="f32", tau=0.7):
    """Adjoint workload: D3Q19 n^3 periodic, random divergence-free start
    (8 Fourier modes |K| <= 4, amplitude 0.02, seed 11), target from seed 12,
    J = 1/2 |u^N - u_tgt|^2.  Times the plain forward (lbm_step), the
    checkpointed forward (lbm_forward_record) and the backward sweep
    (lbm_adjoint: segment recompute + adjoint steps + init map)."""
    import torch

    from paper_2201_11330_amd import lbm
    from paper_2201_11330_amd import workloads as W

    rho, u0 = W.random_fourier_field(n, modes=8, kmax=4, amplitude=0.02, seed=11)
    _, ut0 = W.random_fourier_field(n, modes=8, kmax=4, amplitude=0.02, seed=12)
    tgt = lbm.LBM(lbm.D3Q19, n, n, n, tau, storage=storage)
    tgt.init_equilibrium(rho, ut0)
    tgt.step(steps)
    _, u_tgt = tgt.moments()
    tgt.close()
    sim = lbm.LBM(lbm.D3Q19, n, n, n, tau, storage=storage)
    ckpt = torch.empty((steps // k) * sim.buffer_bytes, dtype=torch.uint8, device="cuda")
    work = torch.empty(lbm.lib().lbm_adjoint_workspace_bytes(sim._h, k), dtype=torch.uint8,
                       device="cuda")

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        out = fn()
        e1.record(sim.stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), out

    for _ in range(2):  # second pass is the measured one
        sim.init_equilibrium(rho, u0)
        t_plain, _ = timed(lambda: sim.step(steps))
        sim.init_equilibrium(rho, u0)
        t_rec, _ = timed(lambda: sim.forward_record(steps, k, ckpt))
        _, uN = sim.moments()
        ubar = (uN - u_tgt).contiguous()
        t_adj, grads = timed(lambda: sim.adjoint(steps, k, ckpt, u0, ubar, work))
    sim.close()
    return {
        "workload": f"D3Q19 {n}^3 periodic, tau={tau}, {steps} steps, checkpoint every {k}, "
                    f"{storage} storage (f - w), random Fourier start",
        "forward_ms": round(t_plain, 3),
        "forward_record_ms": round(t_rec, 3),
        "backward_ms": round(t_adj, 3),
        "backward_over_forward": round(t_adj / t_plain, 3),
        "bytes_model_ratio": 2.5,
        "dJ_dtau": grads[1],
    }


def step_kernel_name(n, storage, pattern):
    """The step kernel liblbm launches for this workload: periodic FP64
    boxes with an even nx and at least 2^20 nodes run two nodes per
    work-item (k_step_ab_pairs, or k_step_aa_even/odd_pairs); FP32 and e4m11
    two-lattice steps of a box whose nx is a power of two from 64 to 4096
    take the row-addressed kernel; everything else one node."""
    if storage == "f64" and n % 2 == 0 and n ** 3 >= 1 << 20:
        return f"k_step_{pattern}_pairs<D3Q19,f64>"
    if storage in ("f32", "e4m11") and pattern == "ab" and 64 <= n <= 4096 and n & (n - 1) == 0:
        return f"k_step_ab_rows<D3Q19,{storage}>"
    return f"k_step_{pattern}<D3Q19,{storage}>"


def kernel_sources_sha256():
    """Hash of everything that decides the code and launch of the step
    kernels: every source of the library (device code, launch plan, store
    policy) and the compiler flags."""
    from paper_2201_11330_amd import build as hip_build

    csrc = os.path.join(ROOT, "paper_2201_11330_amd", "csrc")
    parts = [os.path.join("paper_2201_11330_amd", "csrc", f) for f in sorted(os.listdir(csrc))
             if f.endswith((".hpp", ".hip"))]
    parts.append(os.path.join("include", "lbm.h"))
    h = hashlib.sha256()
    for p in parts:
        h.update(p.encode())
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(hip_build.HIPCC_FLAGS).encode())
    return h.hexdigest()


def build_record():
    """What the timed library was built from and runs on: the in-tree
    library's file hash, the hash of its sources and compiler flags
    (kernel_sources_sha256), the flags, and the device."""
    import torch

    from paper_2201_11330_amd import build as hip_build
    from paper_2201_11330_amd import lbm

    with open(lbm.LIB_PATH, "rb") as fh:
        lib_sha = hashlib.sha256(fh.read()).hexdigest()
    props = torch.cuda.get_device_properties(0)
    return {"library": os.path.relpath(lbm.LIB_PATH, ROOT), "library_sha256": lib_sha,
            "sources_sha256": kernel_sources_sha256(), "hipcc_flags": " ".join(hip_build.HIPCC_FLAGS),
            "device": props.name, "arch": getattr(props, "gcnArchName", None),
            "torch": torch.__version__, "hip": torch.version.hip}


def measured_traffic(storage, pattern, n):
    """HBM bytes per launch of the timed kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE figures (scaled by a plain copy of known size),
    or None when no figures exist for this configuration or the kernel
    sources changed since they were taken."""
    stem = step_kernel_name(n, storage, pattern).split("<")[0]
    path = os.path.join(ROOT, "profiles", f"{stem}_d3q19_{storage}_{n}cube.counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("sources_sha256") != kernel_sources_sha256():
        return None
    return d["traffic_bytes_per_launch"]


def cpu_baseline(n, target_s):
    """The oracle, as it stands, on the host cores: whole-domain steps of the
    same workload, as many as fit in about target_s seconds."""
    import numpy as np

    import oracle
    from paper_2201_11330_amd import workloads as W

    dims = (n, n, n)
    rho, u = W.taylor_green_3d(n, U0=0.05)
    noise = W.population_noise(W.D3Q19, dims, 1e-6, seed=2)
    s = oracle.Sim(oracle.D3Q19, n, n, n, tau=0.6)
    s.init_equilibrium(rho, u, noise)
    del noise
    t0 = time.perf_counter()
    s.step(1)
    t1 = time.perf_counter() - t0
    k = int(max(1, min(50, math.floor(target_s / max(t1, 1e-9)))))
    t0 = time.perf_counter()
    s.step(k)
    dt = time.perf_counter() - t0
    cores = oracle.num_threads()
    # one more step on a single thread, for the per-core rate
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    s.step(1)
    dt1 = time.perf_counter() - t0
    oracle.set_num_threads(cores)
    s.close()
    mlups = n ** 3 * k / dt / 1e6
    return {
        "value": round(mlups, 3),
        "unit": "MLUPS",
        "cores": cores,
        "kind": "oracle",
        "sample": f"D3Q19 {n}^3 FP64 Taylor-Green, {k} whole-domain steps after 1 untimed "
                  f"({dt:.1f} s), AoS paper-order oracle, OpenMP; then 1 step on 1 thread",
        "single_thread_mlups": round(n ** 3 / dt1 / 1e6, 3),
        "cpu_model": host_cpu_model(),
    }


def host_cpu_model():
    """Model name of the host CPU (first entry of /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def line_fp16(args, mlups):
    """FP16 storage (f - w) of the main workload.  Its launches are short
    (~205 us): at least 500 untimed steps (~100 ms) let the clocks settle
    first, and at least 500 timed steps average out their spread."""
    n = args.n
    steps, warmup = max(args.steps, 500), max(args.warmup, 500)
    r = run_gpu(n, "f16", args.pattern, steps, warmup)
    m = n ** 3 * steps / (r["total_ms"] * 1e-3) / 1e6
    a = 2 * 19 * 2 * n ** 3 / (r["launch_ms_mean"] * 1e-3) / 1e9
    return {"kernel": step_kernel_name(n, "f16", args.pattern), "steps": steps, "warmup": warmup,
            "mlups": round(m, 1), "speedup_vs_f64": round(m / mlups, 3) if mlups else None,
            "launch_ms_mean": round(r["launch_ms_mean"], 5), "achieved_gbs": round(a, 1),
            "frac": round(a / HBM_PEAK_GBS, 4)}


def line_compressible(args, mlups):
    n = args.n
    r = run_gpu(n, "f64", args.pattern, args.steps, args.warmup, compressible=True)
    m = n ** 3 * args.steps / (r["total_ms"] * 1e-3) / 1e6
    a = 304 * n ** 3 / (r["launch_ms_mean"] * 1e-3) / 1e9
    return {"workload": "as the main line with the compressible equilibrium of Eq. (feq)",
            "mlups": round(m, 1), "vs_incompressible": round(m / mlups, 3) if mlups else None,
            "launch_ms_mean": round(r["launch_ms_mean"], 5), "achieved_gbs": round(a, 1),
            "frac": round(a / HBM_PEAK_GBS, 4)}


def line_other_pattern(args, mlups):
    n = args.n
    other = "aa" if args.pattern == "ab" else "ab"
    r = run_gpu(n, "f64", other, args.steps, args.warmup)
    m = n ** 3 * args.steps / (r["total_ms"] * 1e-3) / 1e6
    a = 304 * n ** 3 / (r["launch_ms_mean"] * 1e-3) / 1e9
    return {"workload": f"as the main line, {other.upper()} pattern",
            "kernel": step_kernel_name(n, "f64", other), "mlups": round(m, 1),
            "launch_ms_mean": round(r["launch_ms_mean"], 5), "achieved_gbs": round(a, 1),
            "frac": round(a / HBM_PEAK_GBS, 4)}


# Extra lines of the default run, in order (name -> fn(args, main-line MLUPS)).
EXTRA_LINES = {
    "fp16_store": line_fp16,
    "compressible": line_compressible,
    "aa_pattern": line_other_pattern,
    "sustained_256": lambda args, mlups: run_taylor_green_sustained(),
    "precision_512": lambda args, mlups: run_precision(),
    "adjoint": lambda args, mlups: run_adjoint(),
    "channel": lambda args, mlups: run_channel(),
    "channel_sustained": lambda args, mlups: run_channel_sustained(),
    "channel_nodal": lambda args, mlups: run_channel(nodal=True),
    "paper_sphere_d3q27": lambda args, mlups: run_paper_sphere(),
    "small_2d": lambda args, mlups: run_small_2d(),
    "large_2d": lambda args, mlups: run_large_2d(),
}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not built)"}))
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    if args.only:
        print(json.dumps({args.only: EXTRA_LINES[args.only](args, None)}), flush=True)
        return
    n = args.n
    r = run_gpu(n, args.storage, args.pattern, args.steps, args.warmup, args.copy_probe)
    nodes = n ** 3
    mlups = nodes * args.steps / (r["total_ms"] * 1e-3) / 1e6
    blu = 2 * 19 * STORAGE_BYTES[args.storage]
    achieved = blu * nodes / (r["launch_ms_mean"] * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["total_ms"] / args.steps, 5),
        # value and ms_per_step: the K launches and the closing Monitor
        # reduction; roofline: the K launches alone (launch gaps included).
        "timing": {"steps_ms": round(r["launch_ms_mean"] * args.steps, 4),
                   "monitor_ms": round(r["total_ms"] - r["launch_ms_mean"] * args.steps, 4),
                   "mlups_steps_only": round(nodes / (r["launch_ms_mean"] * 1e-3) / 1e6, 1)},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_NAME[args.storage],
        "data": "synthetic",
        "config": {
            "workload": f"D3Q19 {n}^3 periodic 3D Taylor-Green U0=0.05 + 1e-6 noise, tau=0.6, "
                        f"{args.storage} storage, {args.pattern.upper()} fused pull kernel",
            "lattice": "D3Q19", "nx": n, "ny": n, "nz": n, "tau": 0.6,
            "storage": args.storage, "pattern": args.pattern,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.storage, args.pattern, n),
            "kernel": step_kernel_name(n, args.storage, args.pattern),
            "bytes_per_update": blu,
            "launch_ms_mean": round(r["launch_ms_mean"], 5),
        },
        "checks": {"mass_drift": r["mass_drift"], "ke_ratio": r["ke_ratio"],
                   "unstable": r["unstable"]},
    }
    if "copy_probe" in r:
        out["copy_probe"] = r["copy_probe"]
    out["build"] = build_record()
    if not args.no_extras and args.storage == "f64":
        for name, fn in EXTRA_LINES.items():
            out[name] = fn(args, mlups)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

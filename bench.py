"""Throughput of the DISCOS dry step on one MI355X.

Workload: 1,048,576 ions (+1 / -1 halves, z uniform in [a, Lz - a]) on a
256 x 256 x 128 channel, dielectric walls (Neumann limit, sigma = 0), applied field
E_x = 0.1, P3M cutoff 4 h, 9-3 walls, wall-modified dry diffusion, Philox noise.
A step is discos_step: cell list, S^es spread, Poisson (FFT x/y + z tridiagonal),
J^es interpolation, P3M near-field + wall force + dry update.  The same workload also
times the energy / electro-osmotic-flux pass and its hand-written adjoint
(discos_energy_flux, discos_energy_flux_backward) for the adjoint/forward ratio.

The same run times the 512-channel batch, 100 steps of the 65,536-ion dielectric channel
(128 x 128 x 64, E_x = 0.1) and, on the resolved-hydrodynamics channel (262,144 ions,
128^3, charged walls), the wet midpoint step with the Peskin kernel and with the ESC pair
per species.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                [--adjoint-steps A] [--batch-steps B] [--wet-steps S] [--c2-steps S2]
                [--mixed-steps S3]
                [--copy-calibration]
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "dielectric_256x256x128_n1048576"
PROFILED_STEPS = 5  # untimed steps with every stage boundary timed (per-stage breakdown)
METRIC = "ion-timesteps/sec at 1M ions, 256x256x128 grid; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3  # vector FP32 (no matrix cores)

# Algorithmic work per launch of each stage (bytes that the stage must move, or FP64
# flops for the near-field pass), for N ions, C cells and H = (nx/2+1) ny nz
# half-spectrum cells, as the survey prices them.
NEAR_FLOPS_PER_PAIR = 50.0   # FP64 pair work of the P3M correction (pairs within psi, wall
                             # images included)
NEAR_BYTES_PER_ION = 84.0    # the near field's minimum HBM bytes: 36 B read + 48 B written
# peak of the arithmetic each compute-bound stage runs in
ALU_PEAK = {"near_field": FP64_PEAK_TFLOPS}

# Stages that are one kernel launch each, with the kernel's name in rocprofv3 output.
STAGE_KERNEL = {"spread": "spread_charge_kernel", "fft_x": "fft_x_r2c_kernel",
                "z_solve": "zsolve_kernel", "ifft_x": "fft_x_c2r_kernel",
                "interp": "interp_es_kernel", "near_field": "near_field_kernel"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic_dry_step_256x256x128_n1048576.md")
ISSUE_FILE = os.path.join(ROOT, "profiles", "sq_issue_dry_step_256x256x128_n1048576.md")

# The resolved-hydrodynamics channel: wet midpoint step with the random finite
# difference and the stochastic stress, with the 4-point Peskin kernel and with the ESC
# pair of the electro-osmosis runs (App. B: cations w = 7, beta = 7; anions w = 4, beta = 8).
WET_WORKLOAD = "eo_stokes_128x128x128_n262144"
ESC_PAIR = [(7, 7.0), (4, 8.0)]


def gpu_params(p):
    """The GPU side's parameters: p itself.  Both sides read the near-field pair-force
    table from the stored input file (written offline by the oracle's table tool)."""
    return dict(p)


def committed_block(path, kernel):
    """The entry of `kernel` in the fenced JSON block of a committed profile summary (by
    exact name, else the one instantiation of that template), or None if the summary is
    absent or was taken on other sources of that kernel."""
    from paper_2204_14167_amd import rocprof_summary as rs
    try:
        text = open(path).read()
    except OSError:
        return None
    block = text.split("```json", 1)
    if len(block) < 2:
        return None
    data = json.loads(block[1].split("```", 1)[0])
    ks = data.get("kernels", {})
    if kernel in ks:
        name = kernel
    else:
        hits = [k for k in ks if k.split("<", 1)[0] == kernel]
        if len(hits) != 1:
            return None
        name = hits[0]
    return ks[name] if rs.sources_unchanged(data, name) else None


def committed_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter profile (FETCH_SIZE +
    WRITE_SIZE, copy-calibrated), or None if absent or taken on other sources."""
    k = committed_block(TRAFFIC_FILE, kernel)
    return None if k is None else float(k["hbm_bytes_per_launch"])


def committed_issue(kernel):
    """Share of the chip's VALU issue cycles `kernel` fills (SQ instruction counters over
    its kernel-trace duration), or None if absent or taken on other sources."""
    k = committed_block(ISSUE_FILE, kernel)
    return None if k is None else k["valu_issue_share"]


def stage_work(stage, N, C, H, pairs):
    """(bound, algorithmic work, algorithmic HBM bytes) of one launch of a stage."""
    if stage == "cell_list":
        return "hbm", 84.0 * N, 84.0 * N
    if stage == "spread":
        return "hbm", 32.0 * N + 8.0 * C, 32.0 * N + 8.0 * C
    if stage == "fft_x":
        return "hbm", 8.0 * C + 16.0 * H, 8.0 * C + 16.0 * H
    if stage in ("fft_y", "ifft_y", "z_solve"):
        return "hbm", 32.0 * H, 32.0 * H
    if stage == "ifft_x":
        return "hbm", 16.0 * H + 8.0 * C, 16.0 * H + 8.0 * C
    if stage == "interp":
        return "hbm", 56.0 * N + 8.0 * C, 56.0 * N + 8.0 * C
    if stage == "near_list":
        # the padded copy of the sorted ions for the near-field pass: the sorted ion, its
        # bin and permutation entry read (40 B), at least one 52-byte copy written
        return "hbm", 92.0 * N, 92.0 * N
    if stage == "near_field":
        # the pair forces (the candidate tests and the fused dry update are not counted)
        return "alu", NEAR_FLOPS_PER_PAIR * pairs, NEAR_BYTES_PER_ION * N
    # "update": in a dry step the near-field pass applies the update itself (the stage is
    # empty); the hydrodynamic stages are empty too
    return None, None, None


CPU_WORKERS = 16  # host cores of the one-GPU machine


def _oracle_import(_):
    from oracle import dynamics  # noqa: F401  (a worker's imports, before the timing)
    return 0


def _oracle_ion_part(args):
    """The oracle's per-ion part of a dry step for the target ions (a worker process)."""
    from oracle import dynamics, electrostatics as es
    shape, h, pos, q, species, ids, p, targets, pot = args
    grid = es.Grid(*shape, h)
    dynamics.dry_step(grid, pos, q, species, ids, p, 0, targets=targets, near="pairs", pot=pot)
    return len(targets)


def cpu_baseline(w, p, pos, q, ids, species, n_sample=262144):
    """The oracle on the host: its grid part (spread + Poisson) on the whole workload,
    its per-ion part (interpolation, k-d tree near-field, wall force, update) on
    n_sample ions (every ion still sources the fields), extrapolated linearly in the
    ion count to one full step; once on one core, and with the per-ion part split over
    CPU_WORKERS processes (the grid part is numpy's single-threaded FFT either way)."""
    import multiprocessing as mp
    from oracle import dynamics, electrostatics as es
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    t0 = time.perf_counter()
    pot = es.potential(grid, pos, q, p["eps"], p["bc_types"], p["bc_values"])
    t_grid = time.perf_counter() - t0
    targets = np.sort(np.random.default_rng(0).choice(w.n, n_sample, replace=False))
    t0 = time.perf_counter()
    dynamics.dry_step(grid, pos, q, species, ids, p, 0, targets=targets, near="pairs", pot=pot)
    t_ions = time.perf_counter() - t0
    one = w.n / (t_grid + t_ions * w.n / n_sample)
    nw = max(1, min(CPU_WORKERS, os.cpu_count() or 1))
    chunks = np.array_split(targets, nw)
    args = [((w.nx, w.ny, w.nz), w.h, pos, q, species, ids, p, c, pot) for c in chunks]
    # spawned workers: this process has initialised the GPU
    with mp.get_context("spawn").Pool(nw) as pool:
        pool.map(_oracle_import, range(nw), chunksize=1)  # start-up outside the timing
        t0 = time.perf_counter()
        pool.map(_oracle_ion_part, args)
        t_par = time.perf_counter() - t0
    t_step = t_grid + t_par * w.n / n_sample
    return {"value": w.n / t_step, "unit": "ion-timesteps/s", "cores": nw, "kind": "oracle",
            "one_core_value": one,
            "sample": (f"oracle grid part (spread + Poisson) on all {w.n} ions and "
                       f"{w.nx}x{w.ny}x{w.nz} cells ({t_grid:.1f} s, one thread), then the "
                       f"per-ion part of the dry step for {n_sample} sampled ions "
                       f"(interpolation, k-d tree near-field, wall force, update) split over "
                       f"{nw} processes ({t_par:.1f} s; {t_ions:.1f} s on one core), "
                       f"extrapolated linearly to one step of {w.n} ions; numpy / scipy")}


def count_pairs(pos, L, psi, sample=4096):
    """Mean number of neighbours within psi (sampled), for the near-field flop count;
    wall images within psi count as pairs too."""
    rng = np.random.default_rng(1)
    idx = rng.choice(pos.shape[1], sample, replace=False)
    from scipy.spatial import cKDTree
    pts = pos.T.copy()
    tree = cKDTree(pts, boxsize=[L[0], L[1], 1e9])
    cnt = tree.query_ball_point(pts[idx], psi, return_length=True) - 1
    # images below z = 0 (z -> -z) and above z = Lz (z -> 2 Lz - z)
    for zmap in (lambda z: -z, lambda z: 2.0 * L[2] - z):
        img = pts[idx].copy()
        img[:, 2] = zmap(img[:, 2])
        cnt = cnt + tree.query_ball_point(img, psi, return_length=True)
    return float(np.mean(cnt))


def c2_timing(steps, warmup=3):
    """The 65,536-ion dielectric channel (128 x 128 x 64, E_x = 0.1) run for `steps` dry
    steps (its configuration runs 100) after `warmup` untimed ones; inputs in HBM."""
    import torch
    from paper_2204_14167_amd import discos
    import workloads
    w = workloads.WORKLOADS["dielectric_128x128x64_n65536"]
    p = workloads.make_params(w)
    pos, q, ids, species = workloads.make_ions(w)
    ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n)
    dp = ctx.params(gpu_params(p))
    a = [torch.from_numpy(x.copy()).cuda() for x in (pos, q, ids, species)]
    for s in range(warmup):
        ctx.step(*a, dp, s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        ctx.step(*a, dp, warmup + s)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    status = "ok"
    try:
        ctx.check()
    except discos.DiscosError as e:
        status = str(e)
    return {"workload": "dielectric_128x128x64_n65536", "n_ions": w.n, "grid": [w.nx, w.ny, w.nz],
            "steps": steps, "ms_per_step": 1e3 * el / steps,
            "ion_timesteps_per_s": w.n * steps / el, "device_status": status}


def mixed_timing(steps, warmup=2):
    """Walls of mixed type at the size of the 65,536-ion channel: 128 x 128 x 64, the lower
    wall dielectric with a metal strip at 1 kT/e over the middle third of x (the ICEO
    geometry of Sec. IV.B), the upper wall dielectric, E_x = 0.1.  Dry steps (the Poisson
    solve by preconditioned conjugate gradients) and, from steps with stage events, the
    Poisson solve's time."""
    import torch
    from paper_2204_14167_amd import discos
    import workloads
    w0 = workloads.WORKLOADS["dielectric_128x128x64_n65536"]
    w = workloads.Workload("iceo_128x128x64_n65536", w0.nx, w0.ny, w0.nz, w0.n, (1, 1), (0.0, 0.0),
                           e_ext=(0.1, 0.0, 0.0), seed=w0.seed)
    p = workloads.make_params(w)
    strip = np.ones((w.ny, w.nx), dtype=np.int32)  # Neumann (dielectric) columns
    strip[:, w.nx // 3:2 * w.nx // 3] = 0           # Dirichlet (metal) columns
    p["bc_types"] = (strip, 1)
    p["bc_values"] = (np.where(strip == 0, 1.0, 0.0), np.zeros((w.ny, w.nx)))
    pos, q, ids, species = workloads.make_ions(w)
    ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n)
    dp = ctx.params(gpu_params(p))
    a = [torch.from_numpy(x.copy()).cuda() for x in (pos, q, ids, species)]
    for s in range(warmup):
        ctx.step(*a, dp, s)
    ctx.profile(True)
    for s in range(steps):
        ctx.step(*a, dp, warmup + s)
    st = ctx.profile_read()
    ctx.profile(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        ctx.step(*a, dp, warmup + steps + s)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    status = "ok"
    try:
        ctx.check()
    except discos.DiscosError as e:
        status = str(e)
    poisson = sum(st.get(k, 0.0) for k in ("fft_x", "fft_y", "z_solve", "ifft_y", "ifft_x"))
    return {"workload": w.name, "n_ions": w.n, "grid": [w.nx, w.ny, w.nz],
            "walls": "lower: dielectric with a metal strip at 1 kT/e over the middle third of x; "
                     "upper: dielectric",
            "steps": steps, "ms_per_step": 1e3 * el / steps,
            "ion_timesteps_per_s": w.n * steps / el, "poisson_ms": poisson,
            "device_status": status}


def adjoint_timing(ctx, dp, dpos, dq, steps):
    """Mean times of the energy / flux forward pass and of its backward pass (all
    gradients: positions, charges, both wall fields, applied field) on the same
    ions, the backward pass on the forward's cell list as the autograd wrapper runs it;
    ratio = (forward + backward) / forward."""
    import torch
    g = torch.ones(2, dtype=torch.float64, device="cuda")
    out, phi = ctx.energy_flux(dpos, dq, dp)
    ctx.energy_flux_backward(dpos, dq, dp, phi, g, reuse_cells=True)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(steps):
        ctx.energy_flux(dpos, dq, dp, phi=phi, out=out)
    ev[1].record()
    for _ in range(steps):
        ctx.energy_flux_backward(dpos, dq, dp, phi, g, reuse_cells=True)
    ev[2].record()
    torch.cuda.synchronize()
    ctx.check()
    f = ev[0].elapsed_time(ev[1]) / steps
    b = ev[1].elapsed_time(ev[2]) / steps
    return {"forward_ms": f, "backward_ms": b, "ratio": (f + b) / f,
            "gradients": "dU, dQ w.r.t. positions, charges, wall fields, E_ext"}


def wet_stage_bytes(stage, N, C3):
    """Algorithmic bytes of the hydrodynamic stages of one wet step (N ions, C3 face
    values of the three velocity components): S^hy reads positions (32 B), forces
    (24 B) and ids (4 B, the random finite difference) and writes every face once; the
    midpoint J^hy (both gathers by one thread per ion) reads positions (32 B), writes the
    velocity (24 B) and reads the faces once per gather."""
    if stage == "spread_hy":
        return 60.0 * N + 8.0 * C3
    if stage == "interp_hy":
        return 56.0 * N + 16.0 * C3
    return None


def wet_timing(steps, warmup=2):
    """Wet midpoint steps (+ random finite difference, stochastic stress) on the
    resolved-hydrodynamics channel, with the 4-point Peskin kernel, with the ESC pair
    per species, and with the Peskin kernel between two slip walls: ion-timesteps/s and
    per-stage times (hipEvents).

    Every timed step starts from the workload's initial ions (restored by on-device
    copies outside the timed brackets; each step draws new noise).  The workload has no
    ion-ion repulsion, so a few free steps at dt = 0.01 drive close +/- pairs' kicks into
    the 9-3 walls' core, and the wet step carries that unbalanced wall force to every ion
    through the fluid; the model then leaves the stated configuration."""
    import torch
    from paper_2204_14167_amd import discos
    import workloads
    w = workloads.WORKLOADS[WET_WORKLOAD]
    p = workloads.make_params(w)
    p["rfd_delta"] = 1e-4 * w.h
    pos, q, ids, species = workloads.make_ions(w)
    C3 = 3 * w.nx * w.ny * w.nz + w.nx * w.ny
    out = {"workload": WET_WORKLOAD, "n_ions": w.n, "grid": [w.nx, w.ny, w.nz],
           "mode": "wet midpoint step + RFD, stochastic stress, no-slip walls", "steps": steps,
           "timing": ("each step from the initial ions, hipEvents around discos_step; "
                      "per-stage times from as many untimed steps with stage events")}
    for name, kern, slip in (("peskin4", None, (False, False)),
                             ("esc_w7b7_w4b8", ESC_PAIR, (False, False)),
                             ("peskin4_two_slip_walls", None, (True, True))):
        ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n, hydro=True)
        if kern is not None:
            ctx.set_hydro_kernel(kern)
        dp = ctx.params(gpu_params(dict(p, slip=slip)))
        base = [torch.from_numpy(a.copy()).cuda() for a in (pos, q, ids, species)]
        arr = [t.clone() for t in base]
        mode = discos.STEP_WET | discos.STEP_RFD
        for s in range(warmup):
            for a, b in zip(arr, base):
                a.copy_(b)
            ctx.step(*arr, dp, s, mode=mode)
        # per-stage times: steps with an event at every stage boundary (untimed)
        ctx.profile(True)
        for s in range(steps):
            for a, b in zip(arr, base):
                a.copy_(b)
            ctx.step(*arr, dp, warmup + s, mode=mode)
        st = ctx.profile_read()
        ctx.profile(False)
        # timed: hipEvents around each discos_step only
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
        for s in range(steps):
            for a, b in zip(arr, base):
                a.copy_(b)
            ev[2 * s].record()
            ctx.step(*arr, dp, warmup + steps + s, mode=mode)
            ev[2 * s + 1].record()
        torch.cuda.synchronize()
        el = 1e-3 * sum(ev[2 * s].elapsed_time(ev[2 * s + 1]) for s in range(steps))
        ctx.check()
        ctx.close()
        stages = {}
        for k, v in st.items():
            if v <= 0.0:
                continue
            e = {"ms": round(v, 5)}
            b = wet_stage_bytes(k, w.n, C3)
            if b is not None:
                e["GB/s"] = round(b / (v * 1e-3) / 1e9, 1)
                e["hbm_frac"] = round(b / (v * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            stages[k] = e
        out[name] = {"kernels": "4-point Peskin" if kern is None else
                     "ESC (w, beta) = (7, 7) cations, (4, 8) anions",
                     "walls": "slip, slip" if slip[0] else "no-slip, no-slip",
                     "ms_per_step": 1e3 * el / steps, "ion_timesteps_per_s": w.n * steps / el,
                     "stages": stages}
    return out


def batch_timing(steps, seq_steps=3, one_by_one=True):
    """The 512-channel batch (dry steps, uneven grids 16x16x32 .. 64x64x64 and 64 .. 4096
    ions): ion-timesteps/s as one captured graph, as eager batched launches, and with
    the same channels stepped one by one through single-channel contexts."""
    import torch
    from paper_2204_14167_amd import discos
    import workloads
    reps, pos, q, ids, sp = workloads.make_batch(512)
    for r in reps:
        r["mob_coef"] = workloads.batch_channel_params(r)["mob_coef"]
    b = discos.Batch(reps, 1.0, gpu_params(workloads.batch_channel_params(reps[0])))
    arr = [torch.from_numpy(a.copy()).cuda() for a in (pos, q, ids, sp)]
    cfg = b.tune(*arr)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    b.step(*arr, step=0, graph=True)
    b.step(*arr, step=1)
    torch.cuda.synchronize()
    # GPU time per step (events) and the host's time to issue a step (the graph replaces
    # the step's launches by one graph launch; the GPU runs the same kernels either way)
    ev[0].record()
    h0 = time.perf_counter()
    for k in range(steps):
        b.step(*arr, step=2 + k, graph=True)
    h1 = time.perf_counter()
    ev[1].record()
    h2 = time.perf_counter()
    for k in range(steps):
        b.step(*arr, step=2 + steps + k)
    h3 = time.perf_counter()
    ev[2].record()
    torch.cuda.synchronize()
    b.check()
    t_graph = ev[0].elapsed_time(ev[1]) / steps
    t_eager = ev[1].elapsed_time(ev[2]) / steps
    n = pos.shape[1]
    out = {"channels": len(reps), "ions": int(n),
           "cells": int(sum(r["nx"] * r["ny"] * r["nz"] for r in reps)),
           "graph_ms_per_step": t_graph, "eager_ms_per_step": t_eager,
           "host_us_per_step_graph": 1e6 * (h1 - h0) / steps,
           "host_us_per_step_eager": 1e6 * (h3 - h2) / steps,
           "ion_timesteps_per_s_graph": n / (t_graph * 1e-3), "tuned": cfg}
    if not one_by_one:
        return out
    # the same channels one by one (one context per channel, discos_step each)
    ctxs = []
    for r, rep in enumerate(reps):
        w = rep["workload"]
        lo, hi = b.offsets[r], b.offsets[r + 1]
        c = discos.Context(w.nx, w.ny, w.nz, w.h, w.n)
        ctxs.append((c, c.params(gpu_params(workloads.batch_channel_params(rep))),
                     [t[..., lo:hi].contiguous() if t.dim() == 2 else t[lo:hi].clone() for t in arr]))
    for c, prm, a in ctxs:
        c.step(*a, prm, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(seq_steps):
        for c, prm, a in ctxs:
            c.step(*a, prm, 1 + k)
    torch.cuda.synchronize()
    t_seq = 1e3 * (time.perf_counter() - t0) / seq_steps
    out["one_by_one_ms_per_step"] = t_seq
    out["speedup_vs_one_by_one"] = t_seq / t_graph
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=10)
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="steps of the 512-channel batch (0: skip)")
    ap.add_argument("--no-one-by-one", action="store_true",
                    help="skip stepping the batch's channels one by one (keeps kernel traces "
                         "of the batch free of the many small single-channel launches)")
    ap.add_argument("--wet-steps", type=int, default=10,
                    help="wet steps of the 262,144-ion hydrodynamic channel per kernel (0: skip)")
    ap.add_argument("--c2-steps", type=int, default=100,
                    help="timed steps of the 65,536-ion dielectric channel (0: skip)")
    ap.add_argument("--mixed-steps", type=int, default=10,
                    help="dry steps of the 65,536-ion channel with a metal strip on one wall (0: skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of 1 GiB (counter calibration)")
    ap.add_argument("--serial", action="store_true",
                    help="the 1M-ion context runs every stage in order on one stream (each "
                         "kernel alone, for per-kernel profiles); the default overlaps the "
                         "dry step's near field with the grid stages")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the slit-channel step runs on a single MI355X "
              "and is not sharded across GPUs.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2204_14167_amd import discos
    import workloads

    w = workloads.WORKLOADS[WORKLOAD]
    p = workloads.make_params(w)
    pos, q, ids, species = workloads.make_ions(w)
    torch.cuda.set_device(0)
    ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n, serial=args.serial)
    dp = ctx.params(gpu_params(p))
    dpos = torch.from_numpy(pos.copy()).cuda()
    dq = torch.from_numpy(q.copy()).cuda()
    dids = torch.from_numpy(ids.copy()).cuda()
    dsp = torch.from_numpy(species.copy()).cuda()
    for s in range(args.warmup):
        ctx.step(dpos, dq, dids, dsp, dp, s)
    status = []
    try:
        ctx.check()
    except discos.DiscosError as e:
        status.append(f"warmup: {e}")
    # per-stage times from a few steps with an event at every stage boundary (each
    # recorded event costs the stream a few microseconds, so these steps are untimed)
    ctx.profile(True)
    for s in range(PROFILED_STEPS):
        ctx.step(dpos, dq, dids, dsp, dp, args.warmup + s)
    stages = ctx.profile_read()
    ctx.profile(False)
    timed_stages = {k: v for k, v in stages.items() if k in STAGE_KERNEL}
    dom = max(timed_stages, key=timed_stages.get)
    # timed region: only the dominant stage's two events per step, for its live time
    ctx.profile_stages([dom])
    torch.cuda.synchronize()
    first = args.warmup + PROFILED_STEPS
    t0 = time.perf_counter()
    for s in range(args.steps):
        ctx.step(dpos, dq, dids, dsp, dp, first + s)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dom_live_ms = ctx.profile_read()[dom]
    ctx.profile_stages([])
    try:
        ctx.check()
    except discos.DiscosError as e:
        status.append(f"timed: {e}")
    ms_per_step = 1e3 * elapsed / args.steps
    value = w.n * args.steps / elapsed

    adj = adjoint_timing(ctx, dp, dpos, dq, args.adjoint_steps) if args.adjoint_steps > 0 else None
    batched = batch_timing(args.batch_steps, one_by_one=not args.no_one_by_one) if args.batch_steps > 0 else None
    wet = wet_timing(args.wet_steps) if args.wet_steps > 0 else None
    c2 = c2_timing(args.c2_steps) if args.c2_steps > 0 else None
    mixed = mixed_timing(args.mixed_steps) if args.mixed_steps > 0 else None
    if args.copy_calibration:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    N = w.n
    C = w.nx * w.ny * w.nz
    H = (w.nx // 2 + 1) * w.ny * w.nz
    final = dpos.cpu().numpy()
    L = np.array([w.nx, w.ny, w.nz]) * w.h
    pairs = count_pairs(final, L, p["psi"]) * N
    bound, work, abytes = stage_work(dom, N, C, H, pairs)
    t_dom = dom_live_ms * 1e-3
    traffic = committed_traffic(STAGE_KERNEL[dom])
    if bound == "hbm":
        achieved = work / t_dom / 1e9
        roof = {"bound": "hbm", "kernel": STAGE_KERNEL[dom], "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic, "algorithmic_bytes": abytes, "ms_per_launch": dom_live_ms}
    else:
        achieved = work / t_dom / 1e12
        peak = ALU_PEAK[dom]
        roof = {"bound": "alu", "kernel": STAGE_KERNEL[dom], "achieved": achieved,
                "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak, "precision": "fp64",
                "traffic": traffic, "algorithmic_flops": work, "ms_per_launch": dom_live_ms,
                "pairs_per_ion": pairs / N, "flops_per_pair": NEAR_FLOPS_PER_PAIR,
                "algorithmic_bytes": abytes,
                "hbm_GBs_algorithmic": abytes / t_dom / 1e9,
                "hbm_frac_algorithmic": abytes / t_dom / 1e9 / HBM_PEAK_GBS,
                "valu_issue_share": committed_issue(STAGE_KERNEL[dom])}
    roof["traffic_over_algorithmic"] = None if traffic is None else traffic / abytes
    per_stage = {}
    for k, v in stages.items():
        b, wk, ab = stage_work(k, N, C, H, pairs)
        if b is None:
            continue  # empty in a dry step: the update (fused) and the hydrodynamic stages
        e = {"ms": round(v, 5), "bound": b}
        if b == "hbm":
            e["GB/s"] = round(wk / (v * 1e-3) / 1e9, 2)
        else:
            e["TFLOP/s"] = round(wk / (v * 1e-3) / 1e12, 2)
        e["hbm_frac"] = round(ab / (v * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        per_stage[k] = e

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, p, pos, q, ids, species)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "ion-timesteps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n_ions": N, "grid": [w.nx, w.ny, w.nz],
                   "walls": "dielectric (Neumann limit, sigma = 0)", "e_ext": list(w.e_ext),
                   "psi": p["psi"], "mode": "dry step",
                   "streams": "one (serial)" if args.serial else "two (near field beside the grid stages)"},
        "roofline": roof,
        "stages": per_stage,
        "stages_note": (f"per-stage times from {PROFILED_STEPS} untimed steps with an event at every "
                        "stage boundary; the timed steps record only the dominant stage's two "
                        "events (its live launch time in roofline).  " +
                        ("Every stage ran alone (--serial)." if args.serial else
                         "The near field (near_list, near_field) runs on a second stream beside "
                         "spread .. interp, so the stages overlap and do not add up to "
                         "ms_per_step; join_wait is the time the grid stages ran past the "
                         "near-field pass, update the dry update from both forces")),
        "dry_tail": {"join_wait_ms": round(stages.get("interp_hy", 0.0), 5),
                     "update_ms": round(stages.get("update", 0.0), 5)},
        "adjoint_forward_ratio": None if adj is None else adj["ratio"],
        "adjoint": adj,
        "batched": batched,
        "wet": wet,
        "dielectric_128x128x64": c2,
        "mixed_walls": mixed,
        "cpu_baseline": cpu,
        "device_status": "; ".join(status) if status else "ok",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

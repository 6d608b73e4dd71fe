"""Throughput of the DISCOS dry step on one MI355X.

Workload: 1,048,576 ions (+1 / -1 halves, z uniform in [a, Lz - a]) on a
256 x 256 x 128 channel, dielectric walls (Neumann limit, sigma = 0), applied field
E_x = 0.1, P3M cutoff 4 h, 9-3 walls, wall-modified dry diffusion, Philox noise.
A step is discos_step: cell list, S^es spread, Poisson (FFT x/y + z tridiagonal),
J^es interpolation, P3M near-field + wall force + dry update.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
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
METRIC = "ion-timesteps/sec at 1M ions, 256x256x128 grid; adjoint/forward time ratio"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

# Algorithmic work per launch of each stage (bytes that the stage must move, or
# FP64 flops for the compute-bound near-field), for N ions, C cells and H = (nx/2+1) ny nz
# half-spectrum cells.  See the design doc for the derivation.
NEAR_FLOPS_PER_PAIR = 40.0


def stage_work(stage, N, C, H, pairs):
    if stage == "cell_list":
        return "hbm", 84.0 * N
    if stage == "spread":
        return "hbm", 32.0 * N + 8.0 * C
    if stage == "fft_x":
        return "hbm", 8.0 * C + 16.0 * H
    if stage in ("fft_y", "ifft_y", "z_solve"):
        return "hbm", 32.0 * H
    if stage == "ifft_x":
        return "hbm", 16.0 * H + 8.0 * C
    if stage == "interp":
        return "hbm", 56.0 * N + 8.0 * C
    if stage == "near_field":
        return "alu", NEAR_FLOPS_PER_PAIR * pairs
    if stage == "update":
        return "hbm", 104.0 * N
    raise KeyError(stage)


def cpu_baseline(w, p, pos, q, ids, species, n_sample=16):
    """The oracle on the host: its grid part (spread + Poisson) on the whole workload,
    its per-ion part (interpolation, brute-force near-field, update) on n_sample ions,
    extrapolated to one full step."""
    from oracle import dynamics, electrostatics as es
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    t0 = time.perf_counter()
    es.potential(grid, pos, q, p["eps"], p["bc_types"], p["bc_values"])
    t_grid = time.perf_counter() - t0
    targets = np.sort(np.random.default_rng(0).choice(w.n, n_sample, replace=False))
    t0 = time.perf_counter()
    dynamics.dry_step(grid, pos, q, species, ids, p, 0, targets=targets)
    t_sample = time.perf_counter() - t0
    t_ion = max(t_sample - t_grid, 0.0) / n_sample
    t_step = t_grid + t_ion * w.n
    return {"value": w.n / t_step, "unit": "ion-timesteps/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle grid part (spread + Poisson) on all {w.n} ions and "
                       f"{w.nx}x{w.ny}x{w.nz} cells ({t_grid:.1f} s) plus its per-ion part "
                       f"(interpolation, brute-force near-field, update) on {n_sample} ions "
                       f"({t_sample - t_grid:.1f} s), extrapolated to one step of {w.n} ions; "
                       "numpy, single thread")}


def count_pairs(pos, L, psi, sample=4096):
    """Mean number of neighbours within psi (sampled), for the near-field flop count."""
    rng = np.random.default_rng(1)
    idx = rng.choice(pos.shape[1], sample, replace=False)
    from scipy.spatial import cKDTree
    pts = pos.T.copy()
    tree = cKDTree(pts, boxsize=[L[0], L[1], 1e9])
    cnt = tree.query_ball_point(pts[idx], psi, return_length=True) - 1
    return float(np.mean(cnt))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the slit-channel step is measured on a single "
              "MI355X (multi-GPU sharding is a design, not part of this build).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2204_14167_amd import discos, workloads

    w = workloads.WORKLOADS[WORKLOAD]
    p = workloads.make_params(w)
    pos, q, ids, species = workloads.make_ions(w)
    torch.cuda.set_device(0)
    ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n)
    dp = ctx.params(p)
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
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for s in range(args.steps):
        ctx.step(dpos, dq, dids, dsp, dp, args.warmup + s)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = ctx.profile_read()
    ctx.profile(False)
    try:
        ctx.check()
    except discos.DiscosError as e:
        status.append(f"timed: {e}")
    ms_per_step = 1e3 * elapsed / args.steps
    value = w.n * args.steps / elapsed

    N = w.n
    C = w.nx * w.ny * w.nz
    H = (w.nx // 2 + 1) * w.ny * w.nz
    final = dpos.cpu().numpy()
    pairs = count_pairs(final, np.array([w.nx, w.ny, w.nz]) * w.h, p["psi"]) * N
    dom = max(stages, key=stages.get)
    bound, work = stage_work(dom, N, C, H, pairs)
    t_dom = stages[dom] * 1e-3
    if bound == "hbm":
        achieved = work / t_dom / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "algorithmic_bytes": work}
    else:
        achieved = work / t_dom / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                "algorithmic_flops": work, "pairs_per_ion": pairs / N}
    per_stage = {}
    for k, v in stages.items():
        b, wk = stage_work(k, N, C, H, pairs)
        per_stage[k] = {"ms": round(v, 5), "bound": b,
                        ("GB/s" if b == "hbm" else "TFLOP/s"): round(wk / (v * 1e-3) / (1e9 if b == "hbm" else 1e12), 2)}

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
                   "psi": p["psi"], "mode": "dry step"},
        "roofline": roof,
        "stages": per_stage,
        "adjoint_forward_ratio": None,
        "cpu_baseline": cpu,
        "device_status": "; ".join(status) if status else "ok",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Stochastic drift on the GPU (Sec. III, stochastic drift): the equilibrium density of
free particles does not depend on their mobility, so the steps must keep it.
  - Dry step (eq ions3 with the drift D dGamma_z/dz, 9-3 walls): 131,072 uncharged
    particles started from the walls' Boltzmann profile keep it for 1500 steps.
  - Wet step, 100 % wet (eq disc_stokes_temp, midpoint eqs step1 / step2): uncharged
    particles without wall potential stay uniform with the random finite difference of
    eq thermforce, and pile up at the no-slip walls without it (the test has power).
The statistic is the largest deviation over z bins (finest next to the walls) in units
of the binomial standard deviation."""
import numpy as np
import pytest

import workloads
from tests.drift_util import (density_deviation, profile_deviation, sample_wall_profile,
                              wall_profile_bins)
from tests.gpu_util import dev, host, log

pytestmark = pytest.mark.gpu


def _free(nx, ny, nz, n, seed):
    w = workloads.Workload("free", nx, ny, nz, n, (workloads.NEUMANN, workloads.NEUMANN),
                           (0.0, 0.0), seed=seed)
    p = workloads.make_params(w)
    pos, q, ids, sp = workloads.make_ions(w)
    q[:] = 0.0
    return w, p, pos, q, ids, sp


def test_dry_step_keeps_wall_boltzmann_profile():
    from paper_2204_14167_amd import discos
    w, p, pos, q, ids, sp = _free(64, 64, 32, 131072, seed=91)
    rng = np.random.default_rng(92)
    pos[2] = sample_wall_profile(w.n, float(w.nz), p["wall_sigma"], p["wall_xi"], p["wall_cut"], rng)
    prob = wall_profile_bins(float(w.nz), p["wall_sigma"], p["wall_xi"], p["wall_cut"])
    ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n)
    dp = ctx.params(p)
    arrays = (dev(pos), dev(q), dev(ids), dev(sp))
    for s in range(1500):
        ctx.step(*arrays, dp, s)
    ctx.check()
    dmax, ratio = profile_deviation(host(arrays[0])[2], float(w.nz), prob)
    log(f"dry drift: max deviation {dmax:.2f} sigma, ratios {np.round(ratio, 3).tolist()}")
    assert dmax < 5.0


def _wet_run(rfd, steps=1000):
    from paper_2204_14167_amd import discos
    w, p, pos, q, ids, sp = _free(32, 32, 32, 32768, seed=93)
    pos[2] = np.random.default_rng(94).uniform(0.0, float(w.nz), w.n)
    p["wall_on"] = 0
    p["radius"] = np.array([np.inf, np.inf])  # 100 % wet
    p["rfd_delta"] = 1e-4 * w.h if rfd else 0.0
    ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n, hydro=True)
    dp = ctx.params(p)
    mode = discos.STEP_WET | (discos.STEP_RFD if rfd else 0)
    arrays = (dev(pos), dev(q), dev(ids), dev(sp))
    for s in range(steps):
        ctx.step(*arrays, dp, s, mode=mode)
    ctx.check()
    dmax, ratio = density_deviation(host(arrays[0])[2], float(w.nz))
    log(f"wet rfd={rfd}: max deviation {dmax:.2f} sigma, ratios {np.round(ratio, 3).tolist()}")
    return dmax, ratio


def test_wet_step_keeps_uniform_density_with_thermal_forcing():
    dmax, _ = _wet_run(True)
    assert dmax < 5.0


def test_wet_step_without_thermal_forcing_piles_up_at_walls():
    dmax, ratio = _wet_run(False)
    assert dmax > 10.0
    assert ratio[0] > 1.5 and ratio[-1] > 1.5  # excess in the first quarter cell of each wall

"""Pins of the oracle's wet step (CPU only).

  * eq step1 / eq step2 form a midpoint rule: with the noise and the dry terms off,
    one step against an RK4 integration of dx/dt = J(x) v (v frozen) has a local
    error that falls by ~8 per halving of dt (an Euler update, J(x^n) twice or a
    full-step predictor fall by 4);
  * the random finite difference averages to kT div_x S^hy (eq thermforce): the
    mean over many directions of one ion against central differences of S^hy along
    each axis, and its O(delta^2) dependence on the step;
  * with v = 0 (an uncharged ion, no wall force, no noise) the wet step reduces to
    the dry step's Euler-Maruyama update, the dry terms taken at x^n.
"""
import numpy as np
import pytest

from oracle import dynamics, stokes
from oracle.electrostatics import Grid
import workloads


def _setup(n=24, shape=(16, 16, 16), seed=5):
    w = workloads.WORKLOADS["dirichlet_32x32x32_n256"]
    p = workloads.make_params(w)
    nx, ny, nz = shape
    grid = Grid(nx, ny, nz)
    p["bc_types"] = (0, 0)
    p["bc_values"] = (np.zeros((ny, nx)), np.full((ny, nx), 0.5))
    p["e_ext"] = np.array([0.3, 0.0, 0.0])
    pos, q = workloads.random_ions(nx, ny, nz, n, seed)
    pos[2] = 4.0 + (nz - 8.0) * (pos[2] / nz)  # away from the walls
    # the tracked ion (index 0): every coordinate a quarter cell from the kernel kinks
    pos[:, 0] = [5.26, 9.73, 8.24]
    species = (q < 0).astype(np.int32)
    ids = np.arange(n, dtype=np.int64)
    return grid, p, pos, q, species, ids


def _rk4(grid, x, u, v, w, T, m=64):
    h = T / m
    f = lambda y: stokes.interp_velocity(grid, y, u, v, w)
    for _ in range(m):
        k1 = f(x)
        k2 = f(x + 0.5 * h * k1)
        k3 = f(x + 0.5 * h * k2)
        k4 = f(x + h * k3)
        x = x + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return x


def test_midpoint_local_error_is_third_order():
    grid, p, pos, q, species, ids = _setup()
    p["radius"] = np.array([np.inf, np.inf])  # no dry diffusion
    errs = []
    for dt in (0.04, 0.02, 0.01):
        p["dt"] = dt
        new, F, parts = dynamics.wet_step(grid, pos, q, species, ids, p, 0, noise=False,
                                          targets=[0])
        u, v, w = parts["vel"]
        ref = _rk4(grid, pos[:, :1], u, v, w, dt)
        assert np.abs(parts["V0"]).max() * dt < 0.05  # stays inside one kernel piece
        errs.append(np.abs(new - ref).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 6.5 < r1 < 9.5 and 6.5 < r2 < 9.5, (errs, r1, r2)


def test_rfd_mean_is_divergence_of_spreading():
    grid = Grid(8, 8, 8)
    K = 20000
    x = np.array([3.37, 4.81, 1.62])  # near the bottom wall: images contribute
    pos = np.repeat(x[:, None], K, axis=1)
    ids = np.arange(K, dtype=np.int64)
    kT = 1.7
    f = dynamics.thermal_forcing(grid, pos, ids, kT, 1e-4, seed=11, step=2)
    mean = [a / K for a in f]
    # kT div_x S: component c collects d/dx_c of S(x) e_c
    eps = 1e-5
    expect = []
    for c in range(3):
        e = np.zeros((3, 1))
        e[c] = 1.0
        Fc = np.zeros((3, 1))
        Fc[c] = 1.0
        sp = stokes.spread_force(grid, x[:, None] + eps * e, Fc)
        sm = stokes.spread_force(grid, x[:, None] - eps * e, Fc)
        expect.append(kT * (sp[c] - sm[c]) / (2 * eps))
    for c in range(3):
        err = np.linalg.norm(mean[c] - expect[c]) / np.linalg.norm(expect[c])
        assert err < 0.04, (c, err)
    # the other components of the mean vanish only statistically; the exact
    # expectation has no cross terms: check they are small against the diagonal
    assert np.linalg.norm(mean[2][0]) == 0.0 and np.linalg.norm(mean[2][-1]) == 0.0


def test_rfd_step_size_dependence_is_second_order():
    grid = Grid(8, 8, 8)
    # coordinates off the kernel kinks (integers and half-integers in cells)
    pos = np.array([[2.3, 5.7, 6.2], [3.2, 1.2, 7.7], [0.8, 6.3, 4.3]])
    ids = np.arange(3, dtype=np.int64)
    a = dynamics.thermal_forcing(grid, pos, ids, 1.0, 1e-2, 3, 0)
    b = dynamics.thermal_forcing(grid, pos, ids, 1.0, 5e-3, 3, 0)
    c = dynamics.thermal_forcing(grid, pos, ids, 1.0, 2.5e-3, 3, 0)
    d1 = max(np.abs(x - y).max() for x, y in zip(a, b))
    d2 = max(np.abs(x - y).max() for x, y in zip(b, c))
    assert 3.0 < d1 / d2 < 5.0
    scale = max(np.abs(x).max() for x in c)
    assert d2 < 1e-3 * scale


def test_wet_step_with_zero_velocity_is_the_dry_step():
    grid = Grid(16, 16, 16)
    w = workloads.WORKLOADS["dirichlet_32x32x32_n256"]
    p = workloads.make_params(w)
    p["bc_types"] = (0, 0)
    p["bc_values"] = (None, None)
    p["e_ext"] = np.zeros(3)
    pos = np.array([[3.3], [7.1], [8.2]])
    q = np.zeros(1)
    species = np.zeros(1, dtype=np.int32)
    ids = np.array([17], dtype=np.int64)
    new, F, parts = dynamics.wet_step(grid, pos, q, species, ids, p, 4, noise=False)
    assert np.all(F == 0.0) and np.all(parts["V0"] == 0.0)
    dry, _, _ = dynamics.dry_step(grid, pos, q, species, ids, p, 4)
    np.testing.assert_array_equal(new, dry)

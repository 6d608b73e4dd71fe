"""Pins of the oracle's no-slip MAC Stokes path (CPU only).

  * the banded solve satisfies the plain operator definition (residual) and is
    divergence free, for every wall-adjacent row;
  * plane Poiseuille flow: a uniform body force gives the discrete parabola
    f/(2 eta) z (Lz - z) + f h^2/(8 eta) exactly (closed form of the ghost rule);
  * spreading and interpolation are adjoint with the no-slip images and ghosts
    (eq adjoint), and the mobility J L^-1 S is symmetric (eq mob_SHIBA);
  * the stochastic stress obeys the discrete fluctuation-dissipation balance
    exactly: P B B^T P^T = (2 kT / (dV dt)) P with P the solution operator and B
    the noise-to-force map (the identity that fixes the wall-edge variance);
  * the parallel mobility of one particle between the walls follows the analytic
    channel mobility of Sec. III.A for distances >= ~0.7 radii (loose: the
    kernel's effective radius and the periodic images).
"""
import numpy as np
import pytest

from oracle import mobility, stokes
from oracle.electrostatics import Grid
from workloads import random_ions


def _rand_force(grid, seed):
    rng = np.random.default_rng(seed)
    fx = rng.normal(size=(grid.nz, grid.ny, grid.nx))
    fy = rng.normal(size=(grid.nz, grid.ny, grid.nx))
    fz = rng.normal(size=(grid.nz + 1, grid.ny, grid.nx))
    fz[0] = fz[-1] = 0.0
    return fx, fy, fz


@pytest.mark.parametrize("shape", [(8, 8, 8), (4, 8, 5), (16, 4, 6)])
def test_solve_satisfies_operator(shape):
    grid = Grid(*shape, h=0.7)
    fx, fy, fz = _rand_force(grid, sum(shape))
    u, v, w, p = stokes.solve_stokes(grid, 0.37, fx, fy, fz)
    rx, ry, rz, div = stokes.apply_stokes(grid, 0.37, u, v, w, p)
    scale = max(np.abs(fx).max(), np.abs(fz).max())
    assert np.abs(rx - fx).max() < 1e-12 * scale
    assert np.abs(ry - fy).max() < 1e-12 * scale
    assert np.abs(rz[1:-1] - fz[1:-1]).max() < 1e-12 * scale
    assert np.abs(div).max() < 1e-12 * scale
    assert np.all(w[0] == 0) and np.all(w[-1] == 0)
    assert abs(p.mean()) < 1e-12 * np.abs(p).max()


def test_plane_poiseuille_closed_form():
    grid = Grid(8, 4, 12, h=0.5)
    eta, f0 = 0.8, 1.3
    fx = np.full((12, 4, 8), f0)
    fy = np.zeros_like(fx)
    fz = np.zeros((13, 4, 8))
    u, v, w, p = stokes.solve_stokes(grid, eta, fx, fy, fz)
    z = (np.arange(12) + 0.5) * 0.5
    Lz = grid.L[2]
    expect = f0 / (2 * eta) * z * (Lz - z) + f0 * 0.25 / (8 * eta)
    np.testing.assert_allclose(u[:, 2, 3], expect, rtol=1e-12)
    assert np.abs(v).max() < 1e-12 and np.abs(w).max() < 1e-12


def test_spread_interp_adjoint():
    grid = Grid(8, 8, 8)
    pos, _ = random_ions(8, 8, 8, 30, seed=4)
    rng = np.random.default_rng(5)
    pos[2, :10] = rng.uniform(0, 2.0, 10)
    pos[2, 10:20] = 8 - rng.uniform(0, 2.0, 10)
    F = rng.normal(size=(3, 30))
    u, v = rng.normal(size=(2, 8, 8, 8))
    w = rng.normal(size=(9, 8, 8))
    w[0] = w[-1] = 0.0
    fx, fy, fz = stokes.spread_force(grid, pos, F)
    lhs = grid.dV * ((fx * u).sum() + (fy * v).sum() + (fz * w).sum())
    rhs = (F * stokes.interp_velocity(grid, pos, u, v, w)).sum()
    assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + abs(rhs))


def test_mobility_symmetric():
    grid = Grid(8, 8, 8)
    pos = np.array([[1.3, 4.1, 6.6], [2.2, 5.9, 3.3], [0.7, 4.4, 7.2]])
    n = pos.shape[1]
    M = np.zeros((3 * n, 3 * n))
    for col in range(3 * n):
        F = np.zeros((3, n))
        F[col % 3, col // 3] = 1.0
        V, _ = stokes.velocity_at_ions(grid, pos, F, eta=0.5)
        M[:, col] = V.T.reshape(-1)
    np.testing.assert_allclose(M, M.T, atol=1e-13 * np.abs(M).max())
    assert np.all(np.linalg.eigvalsh(0.5 * (M + M.T)) > -1e-13)


def _dense_solution_operator(grid, eta):
    """Columns: velocity (u, v, interior w) for a unit force on each velocity dof."""
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    nu = nz * ny * nx
    nwi = (nz - 1) * ny * nx
    ndof = 2 * nu + nwi
    P = np.zeros((ndof, ndof))
    for col in range(ndof):
        fx = np.zeros((nz, ny, nx))
        fy = np.zeros((nz, ny, nx))
        fz = np.zeros((nz + 1, ny, nx))
        if col < nu:
            fx.reshape(-1)[col] = 1.0
        elif col < 2 * nu:
            fy.reshape(-1)[col - nu] = 1.0
        else:
            fz[1:-1].reshape(-1)[col - 2 * nu] = 1.0
        u, v, w, _ = stokes.solve_stokes(grid, eta, fx, fy, fz)
        P[:, col] = np.concatenate([u.ravel(), v.ravel(), w[1:-1].ravel()])
    return P


def test_fluctuation_dissipation_identity():
    grid = Grid(4, 4, 5, h=0.9)
    eta, kT, dt = 0.6, 1.7, 0.3
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    P = _dense_solution_operator(grid, eta)
    shapes = [(nz, ny, nx)] * 4 + [(nz + 1, ny, nx)] * 2
    sizes = [int(np.prod(s)) for s in shapes]
    amp = np.sqrt(2 * kT * eta / (grid.dV * dt))
    cols = []
    for which, (shp, sz) in enumerate(zip(shapes, sizes)):
        for e in range(sz):
            Ws = [np.zeros(s) for s in shapes]
            Ws[which].reshape(-1)[e] = 1.0
            fx, fy, fz = stokes.stress_divergence(grid, *Ws)
            cols.append(amp * np.concatenate([fx.ravel(), fy.ravel(), fz[1:-1].ravel()]))
    B = np.array(cols).T
    cov = P @ B @ B.T @ P.T
    expect = (2 * kT / (grid.dV * dt)) * P
    assert np.abs(cov - expect).max() < 1e-10 * np.abs(expect).max()


def test_noise_statistics_and_reproducibility():
    grid = Grid(8, 8, 6)
    a = stokes.noise_force(grid, 1.0, 0.5, 0.1, seed=9, step=3)
    b = stokes.noise_force(grid, 1.0, 0.5, 0.1, seed=9, step=3)
    c = stokes.noise_force(grid, 1.0, 0.5, 0.1, seed=9, step=4)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    assert np.abs(a[0] - c[0]).max() > 0
    assert np.all(a[2][0] == 0) and np.all(a[2][-1] == 0)


def test_single_particle_parallel_mobility_near_wall():
    """Parallel mobility of one particle vs the channel formula of Sec. III.A, with
    the 4-point kernel's effective radius measured far from the walls."""
    grid = Grid(32, 32, 32)
    eta = 1.0 / (6 * np.pi)
    heights = [16.0, 4.0, 3.0, 2.0]
    mob = []
    for zz in heights:
        vals = []
        for (x0, y0) in ((10.3, 12.7), (20.8, 5.1)):
            pos = np.array([[x0], [y0], [zz]])
            F = np.array([[1.0], [0.0], [0.0]])
            V, _ = stokes.velocity_at_ions(grid, pos, F, eta)
            vals.append(V[0, 0])
        mob.append(np.mean(vals))
    mob = np.array(mob)
    ratio = mob / mob[0]
    # the same ratio from the analytic channel mobility, radius from the kernel
    # (about 1.25 h for the 4-point Peskin kernel on the MAC grid)
    a = 1.255
    ref = mobility.gamma_channel(np.array(heights), a, 32.0, mobility.PAR)
    ref = ref / ref[0]
    np.testing.assert_allclose(ratio[1:], ref[1:], rtol=0.08)
    assert np.all(np.diff(mob) < 0)  # mobility falls towards the wall

"""Pins of the oracle's slip walls (eq fluidbc: zero normal velocity and zero tangential
stress; Fig. folded: the image spreads the same tangential force), CPU only.

  * closed forms: a uniform body force in a channel with one slip and one no-slip wall
    gives the discrete half-parabola exactly (both orientations); between two slip
    walls a zero-mean cosine force gives the discrete Neumann eigenvector, and a
    uniform force leaves no flow (the kappa = 0 mode's mean force is removed);
  * the solve satisfies the plain operator (with the removed mean force when both
    walls slip) and is divergence free;
  * spreading and interpolation are adjoint with the slip images and ghosts;
  * the stochastic stress obeys the discrete fluctuation-dissipation balance exactly
    with zero stress on slip-wall edges;
  * the mobility is symmetric; an ion on a slip wall keeps tangential but not normal
    velocity, on a no-slip wall neither; the tangential mobility at a slip wall rises
    to about twice its mid-channel value (the ion and its same-sign image coincide)
    while the no-slip one falls to zero.
"""
import numpy as np
import pytest

from oracle import stokes
from oracle.electrostatics import Grid

WALLS = [(True, False), (False, True), (True, True)]


def _rand_force(grid, seed):
    rng = np.random.default_rng(seed)
    fx = rng.normal(size=(grid.nz, grid.ny, grid.nx))
    fy = rng.normal(size=(grid.nz, grid.ny, grid.nx))
    fz = rng.normal(size=(grid.nz + 1, grid.ny, grid.nx))
    fz[0] = fz[-1] = 0.0
    return fx, fy, fz


def test_half_poiseuille_closed_forms():
    grid = Grid(8, 4, 12, h=0.5)
    eta, f0 = 0.8, 1.3
    nz, h = grid.nz, grid.h
    Lz = grid.L[2]
    fx = np.full((nz, 4, 8), f0)
    zero = np.zeros_like(fx)
    fz = np.zeros((nz + 1, 4, 8))
    z = (np.arange(nz) + 0.5) * h
    # no-slip below, slip above: u(0) = 0, u'(Lz) = 0
    u, v, w, _ = stokes.solve_stokes(grid, eta, fx, zero, fz, slip=(False, True))
    expect = f0 / eta * (Lz * z - 0.5 * z * z) + f0 * h * h / (8 * eta)
    np.testing.assert_allclose(u[:, 1, 5], expect, rtol=1e-12)
    assert np.abs(v).max() < 1e-12 and np.abs(w).max() < 1e-12
    # slip below, no-slip above
    u, _, _, _ = stokes.solve_stokes(grid, eta, fx, zero, fz, slip=(True, False))
    expect = f0 / (2 * eta) * (Lz * Lz - z * z) + f0 * h * h / (8 * eta)
    np.testing.assert_allclose(u[:, 2, 0], expect, rtol=1e-12)


def test_two_slip_walls_mean_flow():
    grid = Grid(4, 4, 10, h=0.7)
    eta = 0.45
    nz, h = grid.nz, grid.h
    k = np.arange(nz)
    zero = np.zeros((nz, 4, 4))
    fz = np.zeros((nz + 1, 4, 4))
    for m in (1, 3):
        prof = np.cos(np.pi * m * (k + 0.5) / nz)
        fy = np.broadcast_to(prof[:, None, None], (nz, 4, 4)).copy()
        _, v, _, _ = stokes.solve_stokes(grid, eta, zero, fy, fz, slip=(True, True))
        lam = (2.0 - 2.0 * np.cos(np.pi * m / nz)) / (h * h)
        np.testing.assert_allclose(v[:, 3, 1], prof / (eta * lam), rtol=1e-11, atol=1e-13)
    u, v, w, _ = stokes.solve_stokes(grid, eta, np.full((nz, 4, 4), 2.0), zero, fz,
                                     slip=(True, True))
    assert np.abs(u).max() < 1e-12 and np.abs(v).max() < 1e-12 and np.abs(w).max() < 1e-12


@pytest.mark.parametrize("slip", WALLS)
def test_solve_satisfies_operator(slip):
    grid = Grid(8, 4, 7, h=0.6)
    eta = 0.37
    fx, fy, fz = _rand_force(grid, 5)
    u, v, w, p = stokes.solve_stokes(grid, eta, fx, fy, fz, slip=slip)
    rx, ry, rz, div = stokes.apply_stokes(grid, eta, u, v, w, p, slip=slip)
    ex, ey = fx.copy(), fy.copy()
    if slip[0] and slip[1]:
        # the kappa = 0 tangential force's z-mean is removed
        ex -= fx.mean()
        ey -= fy.mean()
    scale = max(np.abs(fx).max(), np.abs(fz).max())
    assert np.abs(rx - ex).max() < 1e-12 * scale
    assert np.abs(ry - ey).max() < 1e-12 * scale
    assert np.abs(rz[1:-1] - fz[1:-1]).max() < 1e-12 * scale
    assert np.abs(div).max() < 1e-12 * scale
    if slip[0] and slip[1]:
        assert abs(u.mean()) < 1e-12 * np.abs(u).max()


def _wall_ions(grid, n, seed):
    rng = np.random.default_rng(seed)
    L = grid.L
    pos = np.stack([rng.uniform(0, L[0], n), rng.uniform(0, L[1], n), rng.uniform(0, L[2], n)])
    pos[2, : n // 3] = rng.uniform(0, 2.5 * grid.h, n // 3)
    pos[2, n // 3: 2 * n // 3] = L[2] - rng.uniform(0, 2.5 * grid.h, n // 3)
    pos[2, 0], pos[2, 1] = 0.0, L[2]
    return pos


@pytest.mark.parametrize("slip", WALLS)
def test_spread_interp_adjoint(slip):
    grid = Grid(8, 8, 6)
    pos = _wall_ions(grid, 40, 3)
    F = np.random.default_rng(4).normal(size=pos.shape)
    u, v, w = _rand_force(grid, 8)
    sf = stokes.spread_force(grid, pos, F, slip=slip)
    jv = stokes.interp_velocity(grid, pos, u, v, w, slip=slip)
    lhs = sum((a * b).sum() for a, b in zip(sf, (u, v, w))) * grid.dV
    rhs = (F * jv).sum()
    assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + abs(rhs))
    k = np.array([[7, 7.0], [4, 8.0]])[np.arange(pos.shape[1]) % 2]
    sf = stokes.spread_force_kernels(grid, pos, F, k, slip=slip)
    jv = stokes.interp_velocity_kernels(grid, pos, u, v, w, k, slip=slip)
    lhs = sum((a * b).sum() for a, b in zip(sf, (u, v, w))) * grid.dV
    rhs = (F * jv).sum()
    assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + abs(rhs))


def _dense_solution_operator(grid, eta, slip):
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
        u, v, w, _ = stokes.solve_stokes(grid, eta, fx, fy, fz, slip=slip)
        P[:, col] = np.concatenate([u.ravel(), v.ravel(), w[1:-1].ravel()])
    return P


@pytest.mark.parametrize("slip", WALLS)
def test_fluctuation_dissipation_identity(slip):
    grid = Grid(4, 4, 5, h=0.9)
    eta, kT, dt = 0.6, 1.7, 0.3
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    P = _dense_solution_operator(grid, eta, slip)
    np.testing.assert_allclose(P, P.T, atol=1e-12 * np.abs(P).max())
    shapes = [(nz, ny, nx)] * 4 + [(nz + 1, ny, nx)] * 2
    amp = np.sqrt(2 * kT * eta / (grid.dV * dt))
    cols = []
    for which, shp in enumerate(shapes):
        for e in range(int(np.prod(shp))):
            Ws = [np.zeros(s) for s in shapes]
            Ws[which].reshape(-1)[e] = 1.0
            fx, fy, fz = stokes.stress_divergence(grid, *Ws, slip=slip)
            cols.append(amp * np.concatenate([fx.ravel(), fy.ravel(), fz[1:-1].ravel()]))
    B = np.array(cols).T
    cov = P @ B @ B.T @ P.T
    expect = (2 * kT / (grid.dV * dt)) * P
    assert np.abs(cov - expect).max() < 1e-10 * np.abs(expect).max()


def test_wall_velocities_and_mobility():
    grid = Grid(16, 16, 12)
    eta = 1.0 / (6 * np.pi)
    pos = np.array([[5.3, 9.1], [7.7, 3.2], [0.0, 12.0]])  # one ion on each wall
    rng = np.random.default_rng(9)
    F = rng.normal(size=(3, 2))
    for slip in ((True, False), (False, True)):
        V, _ = stokes.velocity_at_ions(grid, pos, F, eta, slip=slip)
        for i, on_slip in ((0, slip[0]), (1, slip[1])):
            assert abs(V[2, i]) < 1e-14 * np.abs(V).max()
            if on_slip:
                assert np.abs(V[:2, i]).min() > 1e-3 * np.abs(V).max()
            else:
                assert np.abs(V[:2, i]).max() < 1e-14 * np.abs(V).max()
    # symmetric mobility with slip walls
    pos3 = np.array([[1.3, 4.1, 6.6], [2.2, 5.9, 3.3], [0.7, 4.4, 7.2]])
    g8 = Grid(8, 8, 8)
    M = np.zeros((9, 9))
    for col in range(9):
        Fc = np.zeros((3, 3))
        Fc[col % 3, col // 3] = 1.0
        V, _ = stokes.velocity_at_ions(g8, pos3, Fc, 0.5, slip=(True, True))
        M[:, col] = V.T.reshape(-1)
    np.testing.assert_allclose(M, M.T, atol=1e-13 * np.abs(M).max())
    assert np.all(np.linalg.eigvalsh(0.5 * (M + M.T)) > -1e-13)


def test_tangential_mobility_near_slip_wall():
    """Fig. folded: the same-sign image keeps the tangential mobility from falling at a
    slip wall.  An ion on the wall and its image coincide, so the fluid carries the
    flow of twice the force mirrored (a half-immersed particle): the mobility rises to
    about twice its mid-channel value, and decreases monotonically away from the wall.
    Next to a no-slip wall it falls to zero."""
    grid = Grid(32, 32, 24)
    eta = 1.0 / (6 * np.pi)
    x0, y0 = 16.3, 15.8

    def par(z, slip):
        F = np.array([[1.0], [0.0], [0.0]])
        V, _ = stokes.velocity_at_ions(grid, np.array([[x0], [y0], [z]]), F, eta, slip=slip)
        return V[0, 0]

    mid = par(12.0, (True, True))
    heights = [0.0, 0.3, 0.6, 1.5, 3.0]
    slip = np.array([par(z, (True, True)) for z in heights]) / mid
    noslip = np.array([par(z, (False, True)) for z in heights]) / mid
    assert 1.8 < slip[0] < 2.3
    assert np.all(np.diff(slip) < 0) and slip[-1] > 1.0
    assert noslip[0] == 0.0 and np.all(np.diff(noslip) > 0)

"""Pins of the oracle's electrostatics on walls whose type varies from column to column
(a metal strip on a dielectric wall, Sec. IV.B; wall data varying along the wall, the
closing remark of Sec. II.B.1), and dense direct solves of every wall pair on grids of
8^3 cells or fewer.

Each pin checks the oracle against something other than itself:
  - a uniform type map reduces every function to the uniform-wall oracle, which has its
    own pins (test_oracle_electrostatics.py);
  - the Poisson solve equals a dense LU solve of the matrix obtained by applying the
    7-point stencil, with ghost layers from ghost_extend, to every unit vector;
  - an affine potential satisfying every column's condition is reproduced exactly;
  - S and J stay adjoint with per-column folds and ghosts;
  - a two-ion configuration is written out by hand from the pair correction;
  - without charges, a grounded wall and a strip at V bound the potential to [0, V].
"""
import numpy as np
import pytest

from oracle import electrostatics as es
from workloads import load_p3m_table, random_ions

D, N = es.DIRICHLET, es.NEUMANN
EPS = 1.0 / (4.0 * np.pi * 4.46)


def _strip_map(nx, ny, lo=None, hi=None, inside=D, outside=N):
    """Type map with `inside` on the columns lo <= i < hi (a strip along y)."""
    lo = nx // 3 if lo is None else lo
    hi = 2 * nx // 3 if hi is None else hi
    t = np.full((ny, nx), outside)
    t[:, lo:hi] = inside
    return t


def _random_map(nx, ny, seed):
    t = np.random.default_rng(seed).integers(0, 2, size=(ny, nx))
    t[0, 0] = D  # a Dirichlet column somewhere: the mixed problem is then nonsingular
    return t


def _apply_operator(grid, eps, types, phi):
    """-eps lap_h phi with homogeneous ghosts, from the ghost-extended array and the
    stencil written out (an assembly independent of poisson_matrix)."""
    ext = es.ghost_extend(grid, eps, types, (None, None), phi, depth=1)
    c = ext[1:-1]
    lap = (np.roll(c, 1, 2) + np.roll(c, -1, 2) + np.roll(c, 1, 1) + np.roll(c, -1, 1)
           + ext[:-2] + ext[2:] - 6.0 * c)
    return -eps * lap / grid.h ** 2


def _dense_matrix(grid, eps, types):
    n = grid.nx * grid.ny * grid.nz
    A = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = _apply_operator(grid, eps, types, e.reshape(grid.nz, grid.ny, grid.nx)).ravel()
    return A


def test_uniform_maps_reduce_to_uniform_walls():
    nx, ny, nz, n = 16, 8, 9, 300
    grid = es.Grid(nx, ny, nz)
    pos, q = random_ions(nx, ny, nz, n, seed=5, charge="normal")
    pos[2, :40] = np.random.default_rng(1).uniform(0.0, 3.0, 40)
    pos[2, 40:80] = nz - np.random.default_rng(2).uniform(0.0, 3.0, 40)
    vals = (np.random.default_rng(3).normal(size=(ny, nx)), np.random.default_rng(4).normal(size=(ny, nx)))
    table, dr = load_p3m_table()
    for bc in ((D, D), (D, N), (N, D), (N, N)):
        maps = (np.full((ny, nx), bc[0]), np.full((ny, nx), bc[1]))
        assert np.array_equal(es.spread_charge(grid, pos, q, maps), es.spread_charge(grid, pos, q, bc))
        assert np.array_equal(es.bc_rhs(grid, EPS, maps, vals), es.bc_rhs(grid, EPS, bc, vals))
        phi = np.random.default_rng(6).normal(size=(nz, ny, nx))
        assert np.array_equal(es.ghost_extend(grid, EPS, maps, vals, phi),
                              es.ghost_extend(grid, EPS, bc, vals, phi))
        rhs = es.spread_charge(grid, pos, q - q.mean(), bc)
        assert np.array_equal(es.solve_poisson(grid, EPS, maps, rhs, project=True),
                              es.solve_poisson(grid, EPS, bc, rhs, project=True))
        assert np.array_equal(es.near_field(grid, pos, q, EPS, 4.0, table, dr, maps),
                              es.near_field(grid, pos, q, EPS, 4.0, table, dr, bc))
        a = es.near_field_pairs(grid, pos, q, EPS, 4.0, table, dr, maps)
        b = es.near_field_pairs(grid, pos, q, EPS, 4.0, table, dr, bc)
        assert np.array_equal(a, b)


@pytest.mark.parametrize("shape", [(8, 8, 8), (8, 4, 5), (4, 8, 7)])
def test_poisson_equals_dense_lu_for_every_wall_pair(shape):
    """Dense direct solves on grids of at most 8^3 cells: uniform wall pairs (the
    all-Neumann pair through the minimum-norm least-squares solution, the oracle's
    gauge), and mixed maps on one or both walls."""
    nx, ny, nz = shape
    grid = es.Grid(nx, ny, nz)
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz)
    cases = [(D, D), (D, N), (N, D), (N, N),
             (_strip_map(nx, ny), N), (N, _strip_map(nx, ny)),
             (_random_map(nx, ny, 1), _random_map(nx, ny, 2)), (_random_map(nx, ny, 3), D)]
    for types in cases:
        A = _dense_matrix(grid, EPS, types)
        rhs = rng.normal(size=(nz, ny, nx))
        if all(np.ndim(t) == 0 for t in types) and types == (N, N):
            rhs -= rhs.mean()
            ref = np.linalg.lstsq(A, rhs.ravel(), rcond=None)[0]
        else:
            ref = np.linalg.solve(A, rhs.ravel())
        got = es.solve_poisson(grid, EPS, types, rhs).ravel()
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_mixed_solve_residual_on_a_larger_grid():
    nx, ny, nz = 16, 16, 12
    grid = es.Grid(nx, ny, nz)
    types = (_strip_map(nx, ny), _random_map(nx, ny, 9))
    rhs = np.random.default_rng(7).normal(size=(nz, ny, nx))
    phi = es.solve_poisson(grid, EPS, types, rhs)
    res = _apply_operator(grid, EPS, types, phi) - rhs
    assert np.abs(res).max() <= 1e-12 * np.abs(rhs).max()


def test_affine_potential_with_mixed_walls():
    """phi = V + E z satisfies a Dirichlet column with phi_b = V (bottom) or V + E Lz
    (top), and a Neumann column with sigma_lo = -eps E, sigma_hi = +eps E (Gauss sign);
    the discrete solution without charges is that affine function exactly."""
    nx, ny, nz, h = 12, 8, 10, 0.5
    grid = es.Grid(nx, ny, nz, h)
    V, E = 0.7, -0.3
    Lz = nz * h
    t_lo, t_hi = _strip_map(nx, ny), _random_map(nx, ny, 11)
    v_lo = np.where(t_lo == D, V, -EPS * E)
    v_hi = np.where(t_hi == D, V + E * Lz, EPS * E)
    rhs = es.bc_rhs(grid, EPS, (t_lo, t_hi), (v_lo, v_hi))
    phi = es.solve_poisson(grid, EPS, (t_lo, t_hi), rhs)
    z = (np.arange(nz) + 0.5) * h
    want = np.broadcast_to((V + E * z)[:, None, None], phi.shape)
    assert np.abs(phi - want).max() <= 1e-12 * np.abs(want).max()
    # the ghosts of the affine function are affine too: E = -E_z everywhere, on every face
    ext = es.ghost_extend(grid, EPS, (t_lo, t_hi), (v_lo, v_hi), phi)
    ex, ey, ez = es.face_fields(grid, ext)
    assert np.abs(ez[1:] + E).max() <= 1e-11
    assert np.abs(ex).max() <= 1e-12 and np.abs(ey).max() <= 1e-12


def test_spread_and_interpolation_stay_adjoint_with_mixed_walls():
    nx, ny, nz, n = 16, 8, 10, 200
    grid = es.Grid(nx, ny, nz)
    pos, q = random_ions(nx, ny, nz, n, seed=21, charge="normal")
    pos[2, :60] = np.random.default_rng(22).uniform(0.0, 2.5, 60)
    pos[2, 60:120] = nz - np.random.default_rng(23).uniform(0.0, 2.5, 60)
    pos[2, 0], pos[2, 1] = 0.0, float(nz)
    types = (_random_map(nx, ny, 24), _strip_map(nx, ny, inside=N, outside=D))
    phi = np.random.default_rng(25).normal(size=(nz, ny, nx))
    rho = es.spread_charge(grid, pos, q, types)
    lhs = grid.dV * np.sum(rho * phi)
    ext = es.ghost_extend(grid, EPS, types, (None, None), phi)
    rhs = np.sum(q * es.interp_scalar(grid, pos, ext))
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + abs(rhs))


def test_near_field_images_take_the_source_column_type():
    """Two ions near the lower wall: A above a dielectric column, B above a metal one.
    The force on each is its pair correction with the other, with the other's image
    (charge of the other's column sign) and with its own image."""
    nx, ny, nz = 16, 16, 16
    grid = es.Grid(nx, ny, nz)
    table, dr = load_p3m_table()
    psi = 4.0
    t_lo = np.full((ny, nx), N)
    t_lo[:, 8:] = D
    pos = np.array([[6.3, 9.1], [5.5, 6.2], [0.8, 1.3]])  # A over column 6 (N), B over 9 (D)
    q = np.array([1.0, -1.0])
    got = es.near_field(grid, pos, q, EPS, psi, table, dr, (t_lo, N))
    img = np.stack([pos[0], pos[1], -pos[2]])
    s = np.array([1.0, -1.0])
    want = np.zeros((3, 2))
    for a in range(2):
        for b in range(2):
            for src, qs in ((pos[:, b], q[b]), (img[:, b], s[b] * q[b])):
                if a == b and src is pos[:, b]:
                    continue
                ok, f = es._pair_force(grid, EPS, psi, table, dr, np.array([q[a]]), np.array([qs]),
                                       (pos[:, a] - src)[:, None])
                if ok[0]:
                    want[:, a] += f[:, 0]
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()
    tgt = es.near_field_pairs(grid, pos, q, EPS, psi, table, dr, (t_lo, N), targets=[0, 1])
    assert np.abs(tgt - want).max() <= 1e-13 * np.abs(want).max()
    allp = es.near_field_pairs(grid, pos, q, EPS, psi, table, dr, (t_lo, N))
    assert np.abs(allp - want).max() <= 1e-13 * np.abs(want).max()


def test_strip_potential_obeys_the_discrete_maximum_principle():
    """No charges, a grounded upper wall, a strip at V on an uncharged dielectric lower
    wall: the solution lies in [0, V], peaks over the strip, and is even about the
    strip's centre."""
    nx, ny, nz = 24, 8, 12
    grid = es.Grid(nx, ny, nz)
    V = 1.5
    t_lo = _strip_map(nx, ny, 8, 16)
    v_lo = np.where(t_lo == D, V, 0.0)
    rhs = es.bc_rhs(grid, EPS, (t_lo, D), (v_lo, None))
    phi = es.solve_poisson(grid, EPS, (t_lo, D), rhs)
    assert phi.min() >= -1e-12 and phi.max() <= V + 1e-12
    assert phi[0, 0, 12] > phi[0, 0, 2]
    # the strip [8, 16) is centred on x = 12: cell i mirrors cell 23 - i
    assert np.abs(phi - phi[:, :, ::-1]).max() <= 1e-11

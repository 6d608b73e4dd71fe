"""GPU parity of the hydrodynamic path: S^hy, the fluctuating no-slip Stokes solve
and J^hy, against the oracle (relative L2 <= 1e-10), plus adjointness on the GPU."""
import numpy as np
import pytest

from oracle import electrostatics as es, shortrange, stokes
import workloads
from tests.gpu_util import TOL, dev, host, log, rel_l2

pytestmark = pytest.mark.gpu


def _ctx(nx, ny, nz, n_max, h=1.0):
    from paper_2204_14167_amd import discos
    return discos.Context(nx, ny, nz, h, n_max, hydro=True)


def _params(eta=1.0 / (6 * np.pi), kT=1.0, dt=0.01, seed=77):
    p = workloads.physical_params()
    p.update(eta=eta, kT=kT, dt=dt, seed=seed, bc_types=(0, 0), bc_values=(None, None),
             e_ext=np.zeros(3))
    return p


def _faces(grid, seed):
    rng = np.random.default_rng(seed)
    fx = rng.normal(size=(grid.nz, grid.ny, grid.nx))
    fy = rng.normal(size=(grid.nz, grid.ny, grid.nx))
    fz = rng.normal(size=(grid.nz + 1, grid.ny, grid.nx))
    fz[0] = fz[-1] = 0.0
    return fx, fy, fz


def _flat(*a):
    return np.concatenate([x.ravel() for x in a])


def _wall_ions(nx, ny, nz, n, seed):
    pos, _ = workloads.random_ions(nx, ny, nz, n, seed)
    rng = np.random.default_rng(seed + 1)
    k = n // 3
    pos[2, :k // 2] = rng.uniform(0, 2.5, k // 2)
    pos[2, k // 2:k] = nz - rng.uniform(0, 2.5, k - k // 2)
    pos[2, 0], pos[2, 1] = 0.0, float(nz)
    return pos


SHAPES = [(16, 16, 16, 400), (32, 8, 10, 700), (8, 16, 20, 300)]


@pytest.mark.parametrize("shape", SHAPES)
def test_spread_force(shape):
    from paper_2204_14167_amd import discos
    nx, ny, nz, n = shape
    log(f"spread_force {shape}")
    grid = es.Grid(nx, ny, nz)
    pos = _wall_ions(nx, ny, nz, n, seed=nx + nz)
    F = np.random.default_rng(2).normal(size=(3, n))
    ref = _flat(*stokes.spread_force(grid, pos, F))
    ctx = _ctx(nx, ny, nz, n)
    out = host(ctx.spread(discos.SPREAD_FORCE, dev(pos), dev(F), ctx.params(_params())))
    assert rel_l2(out, ref) < 1e-13


@pytest.mark.parametrize("shape", [(16, 16, 16), (8, 32, 6), (32, 8, 13), (64, 64, 24)])
def test_stokes_deterministic(shape):
    nx, ny, nz = shape
    log(f"stokes {shape}")
    grid = es.Grid(nx, ny, nz, 0.8)
    fx, fy, fz = _faces(grid, nx + ny + nz)
    u, v, w, p = stokes.solve_stokes(grid, 0.07, fx, fy, fz)
    ctx = _ctx(nx, ny, nz, 1, h=0.8)
    pres = dev(np.zeros((nz, ny, nx)))
    out = host(ctx.solve_stokes(dev(_flat(fx, fy, fz)), ctx.params(_params(eta=0.07)), pres=pres))
    assert rel_l2(out, _flat(u, v, w)) < 1e-11
    assert rel_l2(host(pres), p) < 1e-11
    ctx.check()


def test_stokes_with_stochastic_stress():
    nx, ny, nz = 16, 8, 12
    grid = es.Grid(nx, ny, nz)
    prm = _params(seed=1234)
    fx, fy, fz = _faces(grid, 3)
    nfx, nfy, nfz = stokes.noise_force(grid, prm["kT"], prm["eta"], prm["dt"], prm["seed"], 41)
    u, v, w, p = stokes.solve_stokes(grid, prm["eta"], fx + nfx, fy + nfy, fz + nfz)
    ctx = _ctx(nx, ny, nz, 1)
    out = host(ctx.solve_stokes(dev(_flat(fx, fy, fz)), ctx.params(prm), step=41, noise=True))
    assert rel_l2(out, _flat(u, v, w)) < 1e-11


@pytest.mark.parametrize("shape", SHAPES)
def test_interpolate_velocity(shape):
    from paper_2204_14167_amd import discos
    nx, ny, nz, n = shape
    grid = es.Grid(nx, ny, nz)
    pos = _wall_ions(nx, ny, nz, n, seed=7)
    u, v, w = _faces(grid, 9)
    ref = stokes.interp_velocity(grid, pos, u, v, w)
    ctx = _ctx(nx, ny, nz, n)
    out = host(ctx.interpolate(discos.INTERP_VEL, dev(pos), dev(_flat(u, v, w)), ctx.params(_params())))
    assert rel_l2(out, ref) < 1e-13


def test_hydro_adjointness_on_gpu():
    from paper_2204_14167_amd import discos
    nx, ny, nz, n = 16, 16, 12, 500
    pos = _wall_ions(nx, ny, nz, n, seed=11)
    F = np.random.default_rng(3).normal(size=(3, n))
    u, v, w = _faces(es.Grid(nx, ny, nz), 13)
    ctx = _ctx(nx, ny, nz, n)
    prm = ctx.params(_params())
    sf = host(ctx.spread(discos.SPREAD_FORCE, dev(pos), dev(F), prm))
    jv = host(ctx.interpolate(discos.INTERP_VEL, dev(pos), dev(_flat(u, v, w)), prm))
    lhs = (sf * _flat(u, v, w)).sum()
    rhs = (F * jv).sum()
    assert abs(lhs - rhs) < 1e-13 * (abs(lhs) + abs(rhs))


def test_electro_osmosis_velocity_128cube():
    """The charged-wall set-up on 128^3 with 262,144 ions: forces from the
    electrostatic pass, S^hy, fluctuating no-slip Stokes solve, J^hy."""
    from paper_2204_14167_amd import discos
    w = workloads.WORKLOADS["eo_stokes_128x128x128_n262144"]
    p = workloads.make_params(w)
    pos, q, ids, species = workloads.make_ions(w)
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    log("eo velocity: oracle forces")
    _, _, _, fp = es.grid_force(grid, pos, q, p["eps"], p["bc_types"], p["bc_values"], p["e_ext"])
    F = fp + es.near_field_pairs(grid, pos, q, p["eps"], p["psi"], p["p3m_table"], p["p3m_dr"],
                                 p["bc_types"])
    F[2] += shortrange.wall_force(pos[2], grid.L[2], p["wall_sigma"], p["wall_xi"], p["wall_cut"])
    log("eo velocity: oracle Stokes")
    V_ref, _ = stokes.velocity_at_ions(grid, pos, F, p["eta"], p["kT"], p["dt"], p["seed"], 5)
    log("eo velocity: GPU")
    ctx = _ctx(w.nx, w.ny, w.nz, w.n, w.h)
    dp = ctx.params(p)
    dpos, dq = dev(pos), dev(q)
    rho = ctx.spread(discos.SPREAD_CHARGE | discos.SPREAD_ADD_BC, dpos, dq, dp)
    phi = ctx.solve_poisson(rho, dp)
    Fd = ctx.interpolate(discos.INTERP_FORCE, dpos, phi, dp, aux=dq)
    ctx.near_field(dpos, dq, dp, F=Fd)
    assert rel_l2(host(Fd), F) < TOL
    f = ctx.spread(discos.SPREAD_FORCE, dpos, Fd, dp)
    vel = ctx.solve_stokes(f, dp, step=5, noise=True)
    V = host(ctx.interpolate(discos.INTERP_VEL, dpos, vel, dp))
    ctx.check()
    r = rel_l2(V, V_ref)
    log(f"eo velocity rel-L2 = {r:.3e}")
    assert r < TOL

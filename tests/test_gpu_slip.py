"""GPU parity of slip walls (eq fluidbc, Fig. folded) against the oracle: S^hy and J^hy
with same-sign tangential images, the Stokes solve (deterministic and with the
stochastic stress) for every pair of wall types, wall types changing on one context,
and the wet step with the random finite difference (relative L2 <= 1e-10)."""
import numpy as np
import pytest

from oracle import dynamics, electrostatics as es, stokes
import workloads
from tests.gpu_util import TOL, by_id, dev, host, log, min_image, rel_l2

pytestmark = pytest.mark.gpu

WALLS = [(True, False), (False, True), (True, True), (False, False)]


def _ctx(nx, ny, nz, n_max, h=1.0):
    from paper_2204_14167_amd import discos
    return discos.Context(nx, ny, nz, h, n_max, hydro=True)


def _params(slip, eta=1.0 / (6 * np.pi), kT=1.0, dt=0.01, seed=31):
    p = workloads.physical_params()
    p.update(eta=eta, kT=kT, dt=dt, seed=seed, bc_types=(0, 0), bc_values=(None, None),
             e_ext=np.zeros(3), slip=slip)
    return p


def _faces(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    fz = rng.normal(size=(nz + 1, ny, nx))
    fz[0] = fz[-1] = 0.0
    return rng.normal(size=(nz, ny, nx)), rng.normal(size=(nz, ny, nx)), fz


def _flat(*a):
    return np.concatenate([x.ravel() for x in a])


def _wall_ions(nx, ny, nz, n, seed):
    rng = np.random.default_rng(seed)
    pos = np.stack([rng.uniform(0, nx, n), rng.uniform(0, ny, n), rng.uniform(0, nz, n)])
    k = n // 3
    pos[2, :k // 2] = rng.uniform(0, 4.0, k // 2)
    pos[2, k // 2:k] = nz - rng.uniform(0, 4.0, k - k // 2)
    pos[2, 0], pos[2, 1] = 0.0, float(nz)
    return pos


@pytest.mark.parametrize("slip", WALLS)
def test_spread_and_interp_with_slip(slip):
    from paper_2204_14167_amd import discos
    nx, ny, nz, n = 32, 16, 12, 700
    log(f"slip spread/interp {slip}")
    grid = es.Grid(nx, ny, nz)
    pos = _wall_ions(nx, ny, nz, n, seed=5)
    F = np.random.default_rng(6).normal(size=(3, n))
    u, v, w = _faces(nx, ny, nz, 7)
    ctx = _ctx(nx, ny, nz, n)
    prm = ctx.params(_params(slip))
    sf = host(ctx.spread(discos.SPREAD_FORCE, dev(pos), dev(F), prm))
    assert rel_l2(sf, _flat(*stokes.spread_force(grid, pos, F, slip=slip))) < 1e-13
    jv = host(ctx.interpolate(discos.INTERP_VEL, dev(pos), dev(_flat(u, v, w)), prm))
    assert rel_l2(jv, stokes.interp_velocity(grid, pos, u, v, w, slip=slip)) < 1e-13
    # per-species kernels (the paper's ESC pair) with the same walls
    table = [(7, 7.0), (4, 8.0)]
    sp = (np.arange(n) % 2).astype(np.int32)
    kern = np.asarray(table)[sp]
    ctx.set_hydro_kernel(table)
    sf = host(ctx.spread_species(dev(pos), dev(F), dev(sp), prm))
    assert rel_l2(sf, _flat(*stokes.spread_force_kernels(grid, pos, F, kern, slip=slip))) < TOL
    jv = host(ctx.interpolate_vel_species(dev(pos), dev(_flat(u, v, w)), dev(sp), prm))
    assert rel_l2(jv, stokes.interp_velocity_kernels(grid, pos, u, v, w, kern, slip=slip)) < TOL
    ctx.check()


@pytest.mark.parametrize("slip", WALLS)
@pytest.mark.parametrize("shape", [(16, 16, 12), (32, 8, 7), (8, 16, 40), (8, 8, 160), (8, 8, 300)])
def test_stokes_deterministic_with_slip(slip, shape):
    """Both mode-solve paths: segments of 4 levels per lane, 2 to 64 lanes per mode
    (nz <= 256), and one thread per mode beyond."""
    nx, ny, nz = shape
    log(f"slip stokes {slip} {shape}")
    grid = es.Grid(nx, ny, nz, 0.8)
    fx, fy, fz = _faces(nx, ny, nz, nx + nz)
    u, v, w, p = stokes.solve_stokes(grid, 0.07, fx, fy, fz, slip=slip)
    ctx = _ctx(nx, ny, nz, 1, h=0.8)
    pres = dev(np.zeros((nz, ny, nx)))
    out = host(ctx.solve_stokes(dev(_flat(fx, fy, fz)), ctx.params(_params(slip, eta=0.07)),
                                pres=pres))
    ctx.check()
    assert rel_l2(out, _flat(u, v, w)) < 1e-11
    assert rel_l2(host(pres), p) < 1e-11


@pytest.mark.parametrize("slip", WALLS[:3])
def test_stokes_noise_with_slip(slip):
    nx, ny, nz = 16, 8, 12
    grid = es.Grid(nx, ny, nz)
    prm = _params(slip, seed=4321)
    fx, fy, fz = _faces(nx, ny, nz, 3)
    nfx, nfy, nfz = stokes.noise_force(grid, prm["kT"], prm["eta"], prm["dt"], prm["seed"], 17,
                                       slip=slip)
    u, v, w, _ = stokes.solve_stokes(grid, prm["eta"], fx + nfx, fy + nfy, fz + nfz, slip=slip)
    ctx = _ctx(nx, ny, nz, 1)
    out = host(ctx.solve_stokes(dev(_flat(fx, fy, fz)), ctx.params(prm), step=17, noise=True))
    ctx.check()
    assert rel_l2(out, _flat(u, v, w)) < 1e-11


def test_wall_types_change_on_one_context():
    """The mode factors follow the wall types from call to call."""
    nx, ny, nz = 16, 16, 10
    grid = es.Grid(nx, ny, nz)
    fx, fy, fz = _faces(nx, ny, nz, 11)
    ctx = _ctx(nx, ny, nz, 1)
    f = dev(_flat(fx, fy, fz))
    for slip in [(False, False), (True, True), (True, False), (False, False), (False, True)]:
        u, v, w, _ = stokes.solve_stokes(grid, 0.3, fx, fy, fz, slip=slip)
        out = host(ctx.solve_stokes(f, ctx.params(_params(slip, eta=0.3))))
        assert rel_l2(out, _flat(u, v, w)) < 1e-11, slip
    ctx.check()


@pytest.mark.parametrize("slip", [(True, False), (True, True)])
def test_wet_step_rfd_with_slip(slip):
    from paper_2204_14167_amd import discos
    w = workloads.WORKLOADS["dirichlet_32x32x32_n256"]
    p = workloads.make_params(w)
    p["slip"] = slip
    delta = 1e-4 * w.h
    p["rfd_delta"] = delta
    pos, q, ids, species = workloads.make_ions(w)
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n, hydro=True)
    dp = ctx.params(p)
    args = (dev(pos), dev(q), dev(ids), dev(species))
    log(f"slip wet {slip}: oracle")
    ref, _, _ = dynamics.wet_step(grid, pos, q, species, ids, p, 5, rfd_delta=delta, near="brute")
    log(f"slip wet {slip}: GPU")
    ctx.step(*args, dp, 5, mode=discos.STEP_WET | discos.STEP_RFD)
    ctx.check()
    got = by_id(host(args[0]), host(args[2]), ids)
    r = np.linalg.norm(min_image(got - ref, grid.L)) / np.linalg.norm(min_image(ref - pos, grid.L))
    log(f"slip wet {slip} rel={r:.3e}")
    assert r < TOL


def test_hydro_bc_rejected():
    from paper_2204_14167_amd import discos
    ctx = _ctx(16, 16, 8, 4)
    prm = ctx.params(_params((False, False)))
    prm.struct.hydro_bc[1] = 2
    f = dev(np.zeros(ctx.face_size))
    with pytest.raises(discos.DiscosError, match="hydro_bc"):
        ctx.solve_stokes(f, prm)
    pos = dev(np.array([[1.0], [2.0], [3.0]]))
    with pytest.raises(discos.DiscosError, match="hydro_bc"):
        ctx.spread(discos.SPREAD_FORCE, pos, dev(np.ones((3, 1))), prm)

"""GPU parity of the per-species hydrodynamic kernels (App. B, eq eskernel; the
electro-osmosis runs of Sec. VI give cations the ESC kernel w = 7, beta = 7 and anions
w = 4, beta = 8): S^hy and J^hy with each ion's kernel chosen by its species, and the
wet step with them, against the oracle (relative L2 <= 1e-10)."""
import numpy as np
import pytest

from oracle import dynamics, electrostatics as es, stokes
import workloads
from tests.gpu_util import TOL, by_id, dev, host, log, min_image, rel_l2

pytestmark = pytest.mark.gpu

# kernel tables (w, beta) per species; w = 0 is the 4-point Peskin kernel
KERNELS = {
    # the paper's pair: the widest window (w = 7) takes the 8-node path
    "paper": [(7, 7.0), (4, 8.0)],
    # every kernel within a 4-node window (the 16^3-tile path), Peskin mixed in
    "narrow": [(4, 8.0), (0, 0.0), (3, 5.0), (2, 1.0)],
    # the widest kernel, odd and even widths, beta = 0 (the box kernel), Peskin
    "wide": [(8, 12.0), (5, 4.0), (0, 0.0), (6, 0.0)],
    # the ends of the accepted range: beta = 100 (a sharply peaked kernel, the host
    # quadrature's hardest integrand), the narrowest width, a nearly flat kernel
    "extreme": [(2, 100.0), (8, 100.0), (3, 0.5), (7, 60.0)],
}


def _ctx(nx, ny, nz, n_max, h=1.0):
    from paper_2204_14167_amd import discos
    return discos.Context(nx, ny, nz, h, n_max, hydro=True)


def _params():
    p = workloads.physical_params()
    p.update(eta=1.0 / (6 * np.pi), kT=1.0, dt=0.01, seed=5, bc_types=(0, 0),
             bc_values=(None, None), e_ext=np.zeros(3))
    return p


def _ions(nx, ny, nz, n, nsp, seed, h=1.0):
    """Uniform ions, a third of them within 4 h of a wall (two exactly on the walls),
    species 0 .. nsp (nsp itself: beyond the table, so the Peskin kernel)."""
    rng = np.random.default_rng(seed)
    pos = np.stack([rng.uniform(0, nx * h, n), rng.uniform(0, ny * h, n),
                    rng.uniform(0, nz * h, n)])
    k = n // 3
    pos[2, :k // 2] = rng.uniform(0, 4.0 * h, k // 2)
    pos[2, k // 2:k] = nz * h - rng.uniform(0, 4.0 * h, k - k // 2)
    pos[2, 0], pos[2, 1] = 0.0, nz * h
    sp = rng.integers(0, nsp + 1, n).astype(np.int32)
    return pos, sp


def _per_ion(table, sp):
    t = np.asarray(table, dtype=np.float64).reshape(-1, 2)
    out = np.zeros((len(sp), 2))
    inside = sp < len(t)
    out[inside] = t[sp[inside]]
    return out


def _faces(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    fz = rng.normal(size=(nz + 1, ny, nx))
    fz[0] = fz[-1] = 0.0
    return rng.normal(size=(nz, ny, nx)), rng.normal(size=(nz, ny, nx)), fz


def _flat(*a):
    return np.concatenate([x.ravel() for x in a])


CASES = [("paper", (32, 32, 16, 600)), ("narrow", (32, 16, 12, 500)), ("wide", (16, 32, 12, 500)),
         ("wide", (8, 16, 12, 300)), ("paper", (64, 64, 32, 4096)), ("extreme", (32, 16, 12, 500))]


@pytest.mark.parametrize("kset,shape", CASES)
def test_spread_force_species(kset, shape):
    nx, ny, nz, n = shape
    log(f"esc spread {kset} {shape}")
    table = KERNELS[kset]
    pos, sp = _ions(nx, ny, nz, n, len(table), seed=nx + 3 * nz)
    F = np.random.default_rng(4).normal(size=(3, n))
    grid = es.Grid(nx, ny, nz)
    ref = _flat(*stokes.spread_force_kernels(grid, pos, F, _per_ion(table, sp)))
    ctx = _ctx(nx, ny, nz, n)
    ctx.set_hydro_kernel(table)
    out = host(ctx.spread_species(dev(pos), dev(F), dev(sp), ctx.params(_params())))
    ctx.check()
    r = rel_l2(out, ref)
    log(f"esc spread {kset} {shape} rel={r:.3e}")
    assert r < TOL


@pytest.mark.parametrize("kset,shape", CASES)
def test_interpolate_velocity_species(kset, shape):
    nx, ny, nz, n = shape
    log(f"esc interp {kset} {shape}")
    table = KERNELS[kset]
    pos, sp = _ions(nx, ny, nz, n, len(table), seed=2 * nx + nz)
    u, v, w = _faces(nx, ny, nz, 8)
    grid = es.Grid(nx, ny, nz)
    ref = stokes.interp_velocity_kernels(grid, pos, u, v, w, _per_ion(table, sp))
    ctx = _ctx(nx, ny, nz, n)
    ctx.set_hydro_kernel(table)
    out = host(ctx.interpolate_vel_species(dev(pos), dev(_flat(u, v, w)), dev(sp),
                                           ctx.params(_params())))
    ctx.check()
    r = rel_l2(out, ref)
    log(f"esc interp {kset} {shape} rel={r:.3e}")
    assert r < TOL


def test_species_kernels_adjoint_on_gpu():
    """<S F, v> = <F, J v> with every ion on its own kernel, walls included."""
    nx, ny, nz, n = 32, 16, 14, 800
    table = KERNELS["wide"]
    pos, sp = _ions(nx, ny, nz, n, len(table), seed=17)
    F = np.random.default_rng(5).normal(size=(3, n))
    u, v, w = _faces(nx, ny, nz, 19)
    ctx = _ctx(nx, ny, nz, n)
    ctx.set_hydro_kernel(table)
    prm = ctx.params(_params())
    dsp = dev(sp)
    sf = host(ctx.spread_species(dev(pos), dev(F), dsp, prm))
    jv = host(ctx.interpolate_vel_species(dev(pos), dev(_flat(u, v, w)), dsp, prm))
    lhs = (sf * _flat(u, v, w)).sum()
    rhs = (F * jv).sum()
    assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + abs(rhs))


def test_peskin_rows_and_reset_match_plain_operators():
    """A table of Peskin rows, and a reset table, give the plain S^hy and J^hy."""
    from paper_2204_14167_amd import discos
    nx, ny, nz, n = 16, 16, 10, 300
    pos, sp = _ions(nx, ny, nz, n, 2, seed=3)
    F = np.random.default_rng(6).normal(size=(3, n))
    vel = _flat(*_faces(nx, ny, nz, 7))
    ctx = _ctx(nx, ny, nz, n)
    prm = ctx.params(_params())
    dpos, dF, dsp, dvel = dev(pos), dev(F), dev(sp), dev(vel)
    plain_s = host(ctx.spread(discos.SPREAD_FORCE, dpos, dF, prm))
    plain_j = host(ctx.interpolate(discos.INTERP_VEL, dpos, dvel, prm))
    for tables in ([[(0, 0.0), (0, 3.0)]], [[(7, 7.0)], None]):
        for table in tables:
            ctx.set_hydro_kernel(table)
        assert rel_l2(host(ctx.spread_species(dpos, dF, dsp, prm)), plain_s) < 1e-14
        assert rel_l2(host(ctx.interpolate_vel_species(dpos, dvel, dsp, prm)), plain_j) < 1e-14
    ctx.check()


def _wet(table, rfd, name="dirichlet_32x32x32_n256", edge=False, step=0):
    from paper_2204_14167_amd import discos
    w = workloads.WORKLOADS[name]
    p = workloads.make_params(w)
    p["hydro_kernel"] = np.asarray(table, dtype=np.float64)
    delta = (0.1 if edge else 1e-4) * w.h if rfd else 0.0
    p["rfd_delta"] = delta
    pos, q, ids, species = workloads.make_ions(w)
    if edge:
        # just below the cells a 16^3 face tile gathers without the random finite
        # difference (x0 - 4 for x0 = 16 and 32 = 0): only the shifted w = 8 kernels
        # reach the tile
        rng = np.random.default_rng(43)
        k = np.arange(w.n)
        e = np.where(rng.uniform(size=w.n) < 0.5, 12.0, 28.0) - rng.uniform(1e-4, 0.02, w.n)
        for d in range(3):
            pos[d, k % 3 == d] = e[k % 3 == d]
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n, hydro=True)
    ctx.set_hydro_kernel(table)
    dp = ctx.params(p)
    args = (dev(pos), dev(q), dev(ids), dev(species))
    log(f"esc wet {table} rfd={rfd} edge={edge}: oracle")
    ref, _, _ = dynamics.wet_step(grid, pos, q, species, ids, p, step, rfd_delta=delta,
                                  near="brute")
    log(f"esc wet {table} rfd={rfd} edge={edge}: GPU")
    ctx.step(*args, dp, step, mode=discos.STEP_WET | (discos.STEP_RFD if rfd else 0))
    ctx.check()
    got = by_id(host(args[0]), host(args[2]), ids)
    r = np.linalg.norm(min_image(got - ref, grid.L)) / np.linalg.norm(min_image(ref - pos, grid.L))
    log(f"esc wet rel={r:.3e}")
    assert r < TOL


def test_wet_step_rfd_paper_kernels_eo_128cube():
    """The full-size channel (128^3, 262,144 ions, charged walls) with the paper's pair and
    the random finite difference: one GPU step against the oracle's step at 1,500 sampled
    ions, stored by tests/golden/make_esc_wet_eo128.py (the oracle takes minutes here)."""
    from paper_2204_14167_amd import discos
    from tests.golden import make_esc_wet_eo128 as gold
    w, p, (pos, q, ids, species), targets, delta = gold.case()
    data = np.loadtxt(gold.OUT)
    want = data[:, 0].astype(np.int64)
    ref = data[:, 1:].T
    assert np.array_equal(want, ids[targets])
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n, hydro=True)
    ctx.set_hydro_kernel(gold.KERNELS)
    dp = ctx.params(p)
    args = (dev(pos), dev(q), dev(ids), dev(species))
    log("esc wet eo128: GPU")
    ctx.step(*args, dp, gold.STEP, mode=discos.STEP_WET | discos.STEP_RFD)
    ctx.check()
    got = by_id(host(args[0]), host(args[2]), want)
    old = pos[:, targets]
    r = np.linalg.norm(min_image(got - ref, grid.L)) / np.linalg.norm(min_image(ref - old, grid.L))
    log(f"esc wet eo128 rel={r:.3e}")
    assert r < TOL


def test_wet_step_paper_kernels():
    _wet(KERNELS["paper"], rfd=False)


def test_wet_step_rfd_paper_kernels():
    _wet(KERNELS["paper"], rfd=True, step=2)


def test_wet_step_rfd_widest_kernel_at_tile_edges():
    _wet([(8, 9.0), (4, 8.0)], rfd=True, edge=True, step=3)


def test_full_table_and_out_of_range_species():
    """All DISCOS_HY_MAXSP species set: species outside [0, 8) still take the Peskin
    kernel, not the last species' one."""
    nx, ny, nz, n = 16, 16, 12, 400
    table = [(7, 7.0), (4, 8.0), (5, 3.0), (3, 2.0), (6, 9.0), (2, 1.0), (8, 20.0), (7, 1.5)]
    pos, _ = _ions(nx, ny, nz, n, 8, seed=23)
    sp = np.random.default_rng(24).choice(np.array([-3, -1, 8, 11, 0, 3, 6, 7], dtype=np.int32), n)
    F = np.random.default_rng(25).normal(size=(3, n))
    grid = es.Grid(nx, ny, nz)
    per_ion = np.array([table[k] if 0 <= k < 8 else (0, 0.0) for k in sp], dtype=np.float64)
    ref = _flat(*stokes.spread_force_kernels(grid, pos, F, per_ion))
    ctx = _ctx(nx, ny, nz, n)
    ctx.set_hydro_kernel(table)
    out = host(ctx.spread_species(dev(pos), dev(F), dev(sp), ctx.params(_params())))
    ctx.check()
    assert rel_l2(out, ref) < TOL


def test_hydro_kernel_rejections():
    from paper_2204_14167_amd import discos
    ctx = _ctx(16, 16, 8, 10)
    for bad in ([(9, 5.0)], [(1, 5.0)], [(2.5, 5.0)], [(-2, 5.0)], [(4, -1.0)], [(4, 101.0)],
                [(4, float("nan"))], [(0, 0.0)] * 9):
        with pytest.raises(discos.DiscosError):
            ctx.set_hydro_kernel(bad)
    with pytest.raises(discos.DiscosError, match="nz must exceed"):
        ctx.set_hydro_kernel([(8, 5.0)])
    ctx.set_hydro_kernel([(7, 5.0)])
    ctx.close()
    dry = discos.Context(16, 16, 8, 1.0, 10)
    with pytest.raises(discos.DiscosError, match="HYDRO"):
        dry.set_hydro_kernel([(4, 8.0)])
    dry.close()


def test_species_calls_and_steps_without_ions():
    """n = 0: the species spread returns zero faces, the interpolation and the dry and
    wet steps (with ESC kernels) launch nothing and leave no error."""
    from paper_2204_14167_amd import discos
    w = workloads.WORKLOADS["dirichlet_32x32x32_n256"]
    p = workloads.make_params(w)
    p["rfd_delta"] = 1e-4
    ctx = discos.Context(w.nx, w.ny, w.nz, w.h, 8, hydro=True)
    ctx.set_hydro_kernel(KERNELS["paper"])
    dp = ctx.params(p)
    empty = dev(np.zeros((3, 0)))
    e_sp = dev(np.zeros(0, dtype=np.int32))
    out = host(ctx.spread_species(empty, empty, e_sp, dp))
    assert out.shape == (ctx.face_size,) and np.all(out == 0.0)
    v = dev(np.zeros(ctx.face_size))
    assert host(ctx.interpolate_vel_species(empty, v, e_sp, dp)).shape == (3, 0)
    args = (empty, dev(np.zeros(0)), dev(np.zeros(0, dtype=np.int32)), e_sp)
    ctx.step(*args, dp, 0)
    ctx.step(*args, dp, 1, mode=discos.STEP_WET | discos.STEP_RFD)
    ctx.check()


def test_wet_step_esc_two_slip_walls_rfd():
    """Every addition at once: the paper's ESC pair, two slip walls, the random finite
    difference, one wet step against the oracle's."""
    from paper_2204_14167_amd import discos
    w = workloads.WORKLOADS["dirichlet_32x32x32_n256"]
    p = workloads.make_params(w)
    p["hydro_kernel"] = np.asarray(KERNELS["paper"], dtype=np.float64)
    p["slip"] = (True, True)
    delta = 1e-4 * w.h
    p["rfd_delta"] = delta
    pos, q, ids, species = workloads.make_ions(w)
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n, hydro=True)
    ctx.set_hydro_kernel(KERNELS["paper"])
    args = (dev(pos), dev(q), dev(ids), dev(species))
    ref, _, _ = dynamics.wet_step(grid, pos, q, species, ids, p, 7, rfd_delta=delta, near="brute")
    ctx.step(*args, ctx.params(p), 7, mode=discos.STEP_WET | discos.STEP_RFD)
    ctx.check()
    got = by_id(host(args[0]), host(args[2]), ids)
    r = np.linalg.norm(min_image(got - ref, grid.L)) / np.linalg.norm(min_image(ref - pos, grid.L))
    log(f"esc + two slip walls + rfd rel={r:.3e}")
    assert r < TOL

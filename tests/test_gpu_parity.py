"""GPU parity: the HIP library (through its C ABI) against the oracle, element by
element on the same seeded inputs, at sizes the oracle finishes in seconds that
span several tiles and ragged tails, with ions on and next to the walls.

Bar: relative L2 <= 1e-10 on fields, forces and displacements (the two sides
differ only by FP64 summation order and FMA contraction).
"""
import numpy as np
import pytest

from oracle import dynamics, electrostatics as es, shortrange
import workloads
from tests.gpu_util import TOL, by_id, dev, host, log, min_image, rel_l2

pytestmark = pytest.mark.gpu

D, N = es.DIRICHLET, es.NEUMANN
BC_PAIRS = [(D, D), (N, N), (D, N), (N, D)]
EPS = 1.0 / (4.0 * np.pi * 4.46)


def _ctx(nx, ny, nz, n_max, h=1.0):
    from paper_2204_14167_amd import discos
    return discos.Context(nx, ny, nz, h, n_max)


def _wall_ions(nx, ny, nz, n, seed, h=1.0):
    """Random ions with a third of them within 2.5 h of a wall and two on the walls."""
    pos, q = workloads.random_ions(nx, ny, nz, n, seed, h=h, charge="normal")
    rng = np.random.default_rng(seed + 7)
    k = n // 3
    Lz = nz * h
    pos[2, :k // 2] = rng.uniform(0.0, 2.5 * h, k // 2)
    pos[2, k // 2:k] = Lz - rng.uniform(0.0, 2.5 * h, k - k // 2)
    if n >= 2:
        pos[2, 0] = 0.0
        pos[2, 1] = Lz
    return pos, q


def _params(bc, nx, ny, values=None, eps=EPS, e_ext=(0.0, 0.0, 0.0)):
    p = workloads.physical_params()
    p["eps"] = eps
    p["bc_types"] = bc
    p["bc_values"] = values if values is not None else (None, None)
    p["e_ext"] = np.array(e_ext)
    p["p3m_table"], p["p3m_dr"] = workloads.load_p3m_table()
    return p


SHAPES = [(32, 32, 32, 256), (16, 8, 10, 300), (64, 32, 20, 3000), (8, 16, 37, 500)]


@pytest.mark.parametrize("bc", BC_PAIRS)
@pytest.mark.parametrize("shape", SHAPES)
def test_spread_charge(bc, shape):
    from paper_2204_14167_amd import discos
    nx, ny, nz, n = shape
    log(f"spread bc={bc} shape={shape}")
    pos, q = _wall_ions(nx, ny, nz, n, seed=nx + ny + nz)
    rng = np.random.default_rng(3)
    values = (rng.normal(size=(ny, nx)), rng.normal(size=(ny, nx)))
    p = _params(bc, nx, ny, values)
    grid = es.Grid(nx, ny, nz)
    ref = es.spread_charge(grid, pos, q, bc)
    ctx = _ctx(nx, ny, nz, n)
    dp = ctx.params(p)
    out = host(ctx.spread(discos.SPREAD_CHARGE, dev(pos), dev(q), dp))
    assert rel_l2(out, ref) < 1e-13
    ref_bc = ref + es.bc_rhs(grid, EPS, bc, values)
    out_bc = host(ctx.spread(discos.SPREAD_CHARGE | discos.SPREAD_ADD_BC, dev(pos), dev(q), dp))
    assert rel_l2(out_bc, ref_bc) < 1e-13
    ctx.check()


def test_spread_empty_and_capacity():
    from paper_2204_14167_amd import discos
    ctx = _ctx(16, 16, 8, 10)
    p = ctx.params(_params((D, D), 16, 16))
    out = host(ctx.spread(discos.SPREAD_CHARGE, dev(np.zeros((3, 0))), dev(np.zeros(0)), p))
    assert np.all(out == 0.0)
    pos, q = _wall_ions(16, 16, 8, 11, seed=1)
    with pytest.raises(discos.DiscosError):
        ctx.spread(discos.SPREAD_CHARGE, dev(pos), dev(q), p)


@pytest.mark.parametrize("bc", BC_PAIRS)
@pytest.mark.parametrize("shape", [(32, 32, 32), (8, 16, 5), (64, 8, 12), (256, 16, 4), (16, 128, 9),
                                   (16, 16, 61), (32, 16, 100), (8, 8, 127), (16, 8, 130),
                                   (16, 8, 64), (8, 16, 128), (8, 8, 33), (8, 8, 65)])
def test_poisson(bc, shape):
    nx, ny, nz = shape
    log(f"poisson bc={bc} shape={shape}")
    rhs = np.random.default_rng(nx + 3 * nz).normal(size=(nz, ny, nx))
    if bc == (N, N):
        rhs -= rhs.mean()
    grid = es.Grid(nx, ny, nz, 0.5)
    ref = es.solve_poisson(grid, EPS, bc, rhs)
    ctx = _ctx(nx, ny, nz, 1, h=0.5)
    out = host(ctx.solve_poisson(dev(rhs), ctx.params(_params(bc, nx, ny))))
    assert rel_l2(out, ref) < 1e-12
    ctx.check()


def test_poisson_wall_types_change_on_one_context():
    """The z-solve caches its pivots per wall-type pair: switching types on one context
    must give each problem's own solution."""
    nx, ny, nz = 16, 32, 40
    ctx = _ctx(nx, ny, nz, 1, h=0.5)
    grid = es.Grid(nx, ny, nz, 0.5)
    for k, bc in enumerate([(D, D), (N, N), (D, N), (N, N), (D, D)]):
        rhs = np.random.default_rng(k).normal(size=(nz, ny, nx))
        if bc == (N, N):
            rhs -= rhs.mean()
        ref = es.solve_poisson(grid, EPS, bc, rhs)
        out = host(ctx.solve_poisson(dev(rhs), ctx.params(_params(bc, nx, ny))))
        assert rel_l2(out, ref) < 1e-12, bc
    ctx.check()


def test_poisson_not_neutral_flag():
    from paper_2204_14167_amd import discos
    rhs = np.random.default_rng(5).normal(size=(8, 16, 16))
    rhs += 1.0 - rhs.mean()
    ctx = _ctx(16, 16, 8, 1)
    ctx.solve_poisson(dev(rhs), ctx.params(_params((N, N), 16, 16)))
    with pytest.raises(discos.DiscosError) as e:
        ctx.check()
    assert e.value.code == discos.E_NOT_NEUTRAL
    ctx.check()  # the flag is cleared once reported


@pytest.mark.parametrize("bc", BC_PAIRS)
@pytest.mark.parametrize("shape", [(32, 32, 32, 700), (16, 8, 6, 257)])
def test_interpolate(bc, shape):
    from paper_2204_14167_amd import discos
    nx, ny, nz, n = shape
    log(f"interp bc={bc} shape={shape}")
    rng = np.random.default_rng(11)
    phi = rng.normal(size=(nz, ny, nx))
    values = (rng.normal(size=(ny, nx)), rng.normal(size=(ny, nx)))
    pos, q = _wall_ions(nx, ny, nz, n, seed=5)
    grid = es.Grid(nx, ny, nz)
    p = _params(bc, nx, ny, values, e_ext=(0.1, -0.2, 0.3))
    ext = es.ghost_extend(grid, EPS, bc, values, phi)
    E = es.interp_field(grid, pos, *es.face_fields(grid, ext))
    P = es.interp_scalar(grid, pos, ext)
    ctx = _ctx(nx, ny, nz, n)
    dp = ctx.params(p)
    dpos, dphi = dev(pos), dev(phi)
    assert rel_l2(host(ctx.interpolate(discos.INTERP_E, dpos, dphi, dp)), E) < 1e-13
    F = host(ctx.interpolate(discos.INTERP_FORCE, dpos, dphi, dp, aux=dev(q)))
    assert rel_l2(F, q * (E + np.array([0.1, -0.2, 0.3])[:, None])) < 1e-13
    assert rel_l2(host(ctx.interpolate(discos.INTERP_PHI, dpos, dphi, dp)), P) < 1e-13
    ctx.check()


def test_adjointness_on_gpu():
    """<S q, phi>_h = <q, J phi> (eq adjoint) through the library, walls included."""
    from paper_2204_14167_amd import discos
    nx, ny, nz, n = 32, 16, 24, 2000
    pos, q = _wall_ions(nx, ny, nz, n, seed=21)
    phi = np.random.default_rng(2).normal(size=(nz, ny, nx))
    for bc in BC_PAIRS:
        ctx = _ctx(nx, ny, nz, n)
        dp = ctx.params(_params(bc, nx, ny))
        rho = host(ctx.spread(discos.SPREAD_CHARGE, dev(pos), dev(q), dp))
        jphi = host(ctx.interpolate(discos.INTERP_PHI, dev(pos), dev(phi), dp))
        lhs = (rho * phi).sum()
        rhs = (q * jphi).sum()
        assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + abs(rhs))


@pytest.mark.parametrize("bc", [(D, D), (N, N), (D, N)])
@pytest.mark.parametrize("lj", [False, True])
def test_near_field(bc, lj):
    nx, ny, nz, n = 32, 32, 24, 2500
    log(f"near_field bc={bc} lj={lj}")
    pos, q = _wall_ions(nx, ny, nz, n, seed=9)
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    species = np.where(q > 0, 0, 1).astype(np.int32)
    p = _params(bc, nx, ny)
    if lj:
        p.update(lj_on=True, lj_sigma=np.array([[1.0, 0.8], [0.8, 1.2]]),
                 lj_xi=np.array([[1.0, 2.0], [2.0, 0.5]]), lj_cut_factor=2.5)
    grid = es.Grid(nx, ny, nz)
    ref = es.near_field(grid, pos, q, EPS, p["psi"], p["p3m_table"], p["p3m_dr"], bc)
    ref[2] += shortrange.wall_force(pos[2], grid.L[2], p["wall_sigma"], p["wall_xi"], p["wall_cut"])
    if lj:
        ref += shortrange.lj_pair_forces(grid.L, pos, species, p["lj_sigma"], p["lj_xi"], 2.5)
    keep = np.all(np.isfinite(ref), axis=0)
    ctx = _ctx(nx, ny, nz, n)
    F0 = np.random.default_rng(1).normal(size=(3, n))
    out = host(ctx.near_field(dev(pos), dev(q), ctx.params(p), species=dev(species), F=dev(F0)))
    assert rel_l2((out - F0)[:, keep], ref[:, keep]) < 1e-12


@pytest.mark.parametrize("bc", [(D, N), (N, D)])
@pytest.mark.parametrize("nz", [4, 5, 9, 21])
def test_near_field_channel_heights(bc, nz):
    """Odd heights (the last bin layer is one cell thick, so the images beyond the upper
    wall sit one cell off the bin grid) and channels so thin that an ion's search reaches
    the images of both walls; LJ on, ions on and next to both walls."""
    nx, ny, n = 32, 16, 900
    log(f"near_field heights nz={nz} bc={bc}")
    pos, q = _wall_ions(nx, ny, nz, n, seed=40 + nz)
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    species = np.where(q > 0, 0, 1).astype(np.int32)
    p = _params(bc, nx, ny)
    p.update(lj_on=True, lj_sigma=np.array([[1.0, 0.8], [0.8, 1.2]]),
             lj_xi=np.array([[1.0, 2.0], [2.0, 0.5]]), lj_cut_factor=2.5)
    grid = es.Grid(nx, ny, nz)
    ref = es.near_field(grid, pos, q, EPS, p["psi"], p["p3m_table"], p["p3m_dr"], bc)
    ref[2] += shortrange.wall_force(pos[2], grid.L[2], p["wall_sigma"], p["wall_xi"], p["wall_cut"])
    ref += shortrange.lj_pair_forces(grid.L, pos, species, p["lj_sigma"], p["lj_xi"], 2.5)
    keep = np.all(np.isfinite(ref), axis=0)
    ctx = _ctx(nx, ny, nz, n)
    out = host(ctx.near_field(dev(pos), dev(q), ctx.params(p), species=dev(species)))
    ctx.check()
    assert rel_l2(out[:, keep], ref[:, keep]) < 1e-12


@pytest.mark.parametrize("psi,h,lj_sigma", [
    (1.5, 1.0, None),   # search radius 1 bin (bins of 2 cells)
    (2.0, 1.0, None),   # 1 bin exactly
    (4.5, 1.0, None),   # 3 bins (the LDS copy of the P3M table reaches psi = 5 h)
    (2.4, 0.5, None),   # 3 bins on a finer grid (psi = 4.8 h)
    (4.0, 1.0, 2.0),    # LJ range 5 h beyond psi: 3 bins, LJ pairs past the cutoff
])
def test_near_field_search_radii(psi, h, lj_sigma):
    """The list pass for every search radius it is built for (1 to 3 bins), with ions on
    and near both walls, both wall images, and periodic neighbours across the seams."""
    nx, ny, nz, n = 32, 32, 20, 2000
    bc = (D, N)
    log(f"near_field radii psi={psi} h={h} lj_sigma={lj_sigma}")
    pos, q = _wall_ions(nx, ny, nz, n, seed=13, h=h)
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    species = np.where(q > 0, 0, 1).astype(np.int32)
    p = _params(bc, nx, ny)
    p["psi"] = psi
    if lj_sigma is not None:
        p.update(lj_on=True, lj_sigma=np.full((2, 2), lj_sigma), lj_xi=np.full((2, 2), 0.3),
                 lj_cut_factor=2.5)
    grid = es.Grid(nx, ny, nz, h)
    ref = es.near_field(grid, pos, q, EPS, psi, p["p3m_table"], p["p3m_dr"], bc)
    ref[2] += shortrange.wall_force(pos[2], grid.L[2], p["wall_sigma"], p["wall_xi"], p["wall_cut"])
    if lj_sigma is not None:
        ref += shortrange.lj_pair_forces(grid.L, pos, species, p["lj_sigma"], p["lj_xi"], 2.5)
    keep = np.all(np.isfinite(ref), axis=0)
    ctx = _ctx(nx, ny, nz, n, h=h)
    out = host(ctx.near_field(dev(pos), dev(q), ctx.params(p), species=dev(species)))
    ctx.check()
    assert rel_l2(out[:, keep], ref[:, keep]) < 1e-12


def _step_case(name, steps_checked=1, sample=None, seed_shift=0, near="brute"):
    w = workloads.WORKLOADS[name]
    p = workloads.make_params(w)
    pos, q, ids, species = workloads.make_ions(w)
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    ctx = _ctx(w.nx, w.ny, w.nz, w.n, w.h)
    dp = ctx.params(p)
    dpos, dq, dids, dsp = dev(pos), dev(q), dev(ids), dev(species)
    rng = np.random.default_rng(17)
    for s in range(steps_checked):
        # teacher forcing: both sides start from the GPU's current state
        cur_pos, cur_q, cur_ids, cur_sp = host(dpos), host(dq), host(dids), host(dsp)
        order = np.argsort(cur_ids)
        cur_pos, cur_q, cur_ids, cur_sp = cur_pos[:, order], cur_q[order], cur_ids[order], cur_sp[order]
        targets = None if sample is None else np.sort(rng.choice(w.n, sample, replace=False))
        ref, _, _ = dynamics.dry_step(grid, cur_pos, cur_q, cur_sp, cur_ids, p, s + seed_shift,
                                      targets=targets, near=near)
        ctx.step(dpos, dq, dids, dsp, dp, s + seed_shift)
        ctx.check()
        got_all, got_ids = host(dpos), host(dids)
        want = cur_ids if targets is None else cur_ids[targets]
        got = by_id(got_all, got_ids, want)
        old = cur_pos if targets is None else cur_pos[:, targets]
        err = min_image(got - ref, grid.L)
        disp = min_image(ref - old, grid.L)
        r = np.linalg.norm(err) / np.linalg.norm(disp)
        log(f"step {name} s={s} rel={r:.3e}")
        assert r < TOL
        # the arrays stay a permutation of the ions
        assert np.array_equal(np.sort(got_ids), np.arange(w.n))
        assert np.array_equal(host(dq)[np.argsort(got_ids)], q)


def test_step_grounded_32cube():
    _step_case("dirichlet_32x32x32_n256", steps_checked=3)


def test_step_dielectric_32cube():
    _step_case("dielectric_32x32x32_n4096", steps_checked=2, sample=600)


def test_step_dielectric_128x128x64():
    _step_case("dielectric_128x128x64_n65536", steps_checked=2, sample=400)


def test_step_dielectric_128x128x64_100_steps():
    """The 65,536-ion dielectric channel with E_x = 0.1 run for its 100 steps on the GPU.
    Every 10th step is checked teacher-forced: the oracle takes the GPU's state before the
    step and computes the step for 400 sampled ions (near field by the oracle's k-d tree
    route, pinned against its brute-force sum), which must agree to 1e-10."""
    w = workloads.WORKLOADS["dielectric_128x128x64_n65536"]
    assert w.steps == 100
    p = workloads.make_params(w)
    pos, q, ids, species = workloads.make_ions(w)
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    ctx = _ctx(w.nx, w.ny, w.nz, w.n, w.h)
    dp = ctx.params(p)
    dpos, dq, dids, dsp = dev(pos), dev(q), dev(ids), dev(species)
    rng = np.random.default_rng(29)
    for s in range(w.steps):
        if s % 10 == 0:
            cur_pos, cur_q, cur_ids, cur_sp = host(dpos), host(dq), host(dids), host(dsp)
            order = np.argsort(cur_ids)
            cur_pos, cur_q, cur_ids, cur_sp = cur_pos[:, order], cur_q[order], cur_ids[order], cur_sp[order]
            targets = np.sort(rng.choice(w.n, 400, replace=False))
            ref, _, _ = dynamics.dry_step(grid, cur_pos, cur_q, cur_sp, cur_ids, p, s, targets=targets,
                                          near="pairs")
        ctx.step(dpos, dq, dids, dsp, dp, s)
        if s % 10 == 0:
            ctx.check()
            got = by_id(host(dpos), host(dids), cur_ids[targets])
            err = min_image(got - ref, grid.L)
            disp = min_image(ref - cur_pos[:, targets], grid.L)
            r = np.linalg.norm(err) / np.linalg.norm(disp)
            log(f"c2 step {s}: rel {r:.3e}")
            assert r < TOL
    ctx.check()
    got_pos, got_ids = host(dpos), host(dids)
    assert np.all(np.isfinite(got_pos))
    assert np.array_equal(np.sort(got_ids), np.arange(w.n))
    assert np.all((got_pos[2] >= 0.0) & (got_pos[2] <= grid.L[2]))


def test_step_headline_1m_sampled():
    """The timed workload itself: 1,048,576 ions on 256x256x128 with dielectric walls and
    E_x = 0.1, one step in the library's launch configuration, against the oracle at
    1,500 sampled ions (the oracle's near field from its pair search; about 16 s)."""
    _step_case("dielectric_256x256x128_n1048576", steps_checked=1, sample=1500, near="pairs")


def test_near_field_dense_cluster():
    """A cluster denser than a workgroup's LDS stage holds: that block takes the
    global-memory path; results must not change."""
    nx, ny, nz, n = 32, 32, 16, 3000
    rng = np.random.default_rng(12)
    pos = np.empty((3, n))
    pos[0] = rng.uniform(10.0, 16.0, n)
    pos[1] = rng.uniform(10.0, 16.0, n)
    pos[2] = rng.uniform(0.2, 6.0, n)
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    p = _params((D, N), nx, ny)
    grid = es.Grid(nx, ny, nz)
    ref = es.near_field(grid, pos, q, EPS, p["psi"], p["p3m_table"], p["p3m_dr"], (D, N))
    ref[2] += shortrange.wall_force(pos[2], grid.L[2], p["wall_sigma"], p["wall_xi"], p["wall_cut"])
    ctx = _ctx(nx, ny, nz, n)
    out = host(ctx.near_field(dev(pos), dev(q), ctx.params(p)))
    assert rel_l2(out, ref) < 1e-12


@pytest.mark.parametrize("bc", [(D, D), (N, N)])
def test_near_field_cutoff_and_coincidence_edges(bc):
    """Pairs just inside / just outside the cutoff far from the origin of a wide box
    (where FP32 positions are coarsest), a pair closer than the FP32 resolution, a
    coincident pair and an ion on a wall: the FP32 candidate filter keeps every pair
    inside the cutoff, the exact FP64 test decides, zero separations contribute nothing."""
    nx, ny, nz = 1024, 16, 24
    psi = 4.0
    pts, qs = [], []
    rng = np.random.default_rng(31)
    for k in range(40):  # pairs at psi -/+ 1e-9 along random directions, x near 1000
        c = np.array([1000.0 + rng.uniform(-10, 10), rng.uniform(0, 16), rng.uniform(6, 18)])
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r = psi - 1e-9 if k % 2 == 0 else psi + 1e-9
        pts += [c, c + r * d]
        qs += [1.0, -1.0]
    c = np.array([1017.3, 5.5, 12.0])
    pts += [c, c + np.array([1e-7, 0.0, 0.0])]  # distinct in FP64, equal in FP32
    qs += [1.0, 1.0]
    pts += [np.array([3.0, 7.0, 9.0])] * 2       # coincident
    qs += [1.0, -1.0]
    pts += [np.array([500.0, 3.0, 0.0]), np.array([501.5, 3.0, 24.0])]  # on the walls
    qs += [1.0, -1.0]
    pos = np.array(pts).T.copy()
    pos[0] %= nx
    q = np.array(qs)
    p = _params(bc, nx, ny)
    grid = es.Grid(nx, ny, nz)
    ref = es.near_field(grid, pos, q, EPS, psi, p["p3m_table"], p["p3m_dr"], bc)
    ref[2] += shortrange.wall_force(pos[2], grid.L[2], p["wall_sigma"], p["wall_xi"], p["wall_cut"])
    ctx = _ctx(nx, ny, nz, pos.shape[1])
    out = host(ctx.near_field(dev(pos), dev(q), ctx.params(p)))
    assert np.all(np.isfinite(out))
    assert rel_l2(out, ref) < 1e-12


@pytest.mark.parametrize("name", ["dielectric_32x32x32_n4096", "dielectric_128x128x64_n65536"])
def test_step_serial_equals_two_streams(name):
    """A context created with DISCOS_CREATE_SERIAL (every stage in order on the caller's
    stream, the update inside the near-field pass) and one whose dry step runs the near
    field on its second stream give the same steps: per ion the same forces summed in
    the same order, so equal to rounding of the in-bin order of the cell list."""
    from paper_2204_14167_amd import discos
    w = workloads.WORKLOADS[name]
    p = workloads.make_params(w)
    pos, q, ids, species = workloads.make_ions(w)
    out = []
    for serial in (True, False):
        ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n, serial=serial)
        dp = ctx.params(p)
        arrays = (dev(pos), dev(q), dev(ids), dev(species))
        for s in range(3):
            ctx.step(*arrays, dp, s)
        ctx.check()
        out.append(by_id(host(arrays[0]), host(arrays[2]), np.arange(w.n)))
    L = np.array([w.nx, w.ny, w.nz], float) * w.h
    rel = np.linalg.norm(min_image(out[0] - out[1], L)) / np.linalg.norm(min_image(out[0] - pos, L))
    log(f"{name}: serial vs two streams over 3 steps, rel {rel:.3e}")
    assert rel < 1e-12

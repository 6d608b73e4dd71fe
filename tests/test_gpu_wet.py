"""GPU parity of the wet step (eq disc_stokes_temp, eq step1, eq step2, optional
thermal forcing of eq thermforce) against the oracle's wet step: displacements to
relative L2 <= 1e-10, both sides starting from the same state each step."""
import numpy as np
import pytest

from oracle import dynamics, electrostatics as es
import workloads
from tests.gpu_util import TOL, by_id, dev, host, log, min_image

pytestmark = pytest.mark.gpu


def _ctx(w):
    from paper_2204_14167_amd import discos
    return discos.Context(w.nx, w.ny, w.nz, w.h, w.n, hydro=True)


def _wet_case(name, steps_checked=1, sample=None, rfd=False, pure_wet=False, seed_shift=0,
              slip=None):
    from paper_2204_14167_amd import discos
    w = workloads.WORKLOADS[name]
    p = workloads.make_params(w)
    if pure_wet:
        p["radius"] = np.array([np.inf, np.inf])
    delta = 1e-4 * w.h if rfd else 0.0
    p["rfd_delta"] = delta
    if slip is not None:
        p["slip"] = slip
    pos, q, ids, species = workloads.make_ions(w)
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    ctx = _ctx(w)
    dp = ctx.params(p)
    mode = discos.STEP_WET | (discos.STEP_RFD if rfd else 0)
    dpos, dq, dids, dsp = dev(pos), dev(q), dev(ids), dev(species)
    rng = np.random.default_rng(23)
    near = "brute" if w.n <= 1024 else "pairs"
    for s in range(steps_checked):
        cur_pos, cur_q, cur_ids, cur_sp = host(dpos), host(dq), host(dids), host(dsp)
        order = np.argsort(cur_ids)
        cur_pos, cur_q, cur_ids, cur_sp = cur_pos[:, order], cur_q[order], cur_ids[order], cur_sp[order]
        targets = None if sample is None else np.sort(rng.choice(w.n, sample, replace=False))
        log(f"wet {name} rfd={rfd} s={s}: oracle")
        ref, _, _ = dynamics.wet_step(grid, cur_pos, cur_q, cur_sp, cur_ids, p, s + seed_shift,
                                      rfd_delta=delta, near=near, targets=targets)
        log(f"wet {name} rfd={rfd} s={s}: GPU")
        ctx.step(dpos, dq, dids, dsp, dp, s + seed_shift, mode=mode)
        ctx.check()
        got_all, got_ids = host(dpos), host(dids)
        want = cur_ids if targets is None else cur_ids[targets]
        got = by_id(got_all, got_ids, want)
        old = cur_pos if targets is None else cur_pos[:, targets]
        err = min_image(got - ref, grid.L)
        disp = min_image(ref - old, grid.L)
        r = np.linalg.norm(err) / np.linalg.norm(disp)
        log(f"wet {name} rfd={rfd} s={s} rel={r:.3e}")
        assert r < TOL
        assert np.array_equal(np.sort(got_ids), np.arange(w.n))
        assert np.array_equal(host(dq)[np.argsort(got_ids)], q)


def test_wet_step_grounded_32cube():
    _wet_case("dirichlet_32x32x32_n256", steps_checked=2)


def test_wet_step_rfd_grounded_32cube():
    _wet_case("dirichlet_32x32x32_n256", steps_checked=2, rfd=True, seed_shift=5)


def test_pure_wet_step_32cube():
    _wet_case("dirichlet_32x32x32_n256", steps_checked=1, pure_wet=True)


def test_wet_step_rfd_dielectric_32cube():
    _wet_case("dielectric_32x32x32_n4096", steps_checked=1, sample=600, rfd=True)


def test_wet_step_electro_osmosis_128cube():
    _wet_case("eo_stokes_128x128x128_n262144", steps_checked=1, sample=1500)


def test_wet_step_rfd_electro_osmosis_128cube():
    """The timed no-slip variant with the random finite difference, 1,500 sampled ions."""
    _wet_case("eo_stokes_128x128x128_n262144", steps_checked=1, sample=1500, rfd=True,
              seed_shift=3)


def test_wet_step_rfd_two_slip_walls_128cube():
    """The timed slip-wall variant: 262,144 ions on 128^3 between two slip walls, with the
    random finite difference, at 1,500 sampled ions."""
    _wet_case("eo_stokes_128x128x128_n262144", steps_checked=1, sample=1500, rfd=True,
              slip=(True, True), seed_shift=7)


def test_wet_step_rejections():
    from paper_2204_14167_amd import discos
    w = workloads.WORKLOADS["dirichlet_32x32x32_n256"]
    p = workloads.make_params(w)
    pos, q, ids, species = workloads.make_ions(w)
    args = (dev(pos), dev(q), dev(ids), dev(species))
    dry_ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n)
    with pytest.raises(discos.DiscosError, match="HYDRO"):
        dry_ctx.step(*args, dry_ctx.params(p), 0, mode=discos.STEP_WET)
    ctx = _ctx(w)
    with pytest.raises(discos.DiscosError, match="needs DISCOS_STEP_WET"):
        ctx.step(*args, ctx.params(p), 0, mode=discos.STEP_RFD)
    for bad in (0.0, 0.2 * w.h, float("nan")):
        p["rfd_delta"] = bad
        with pytest.raises(discos.DiscosError, match="rfd_delta"):
            ctx.step(*args, ctx.params(p), 0, mode=discos.STEP_WET | discos.STEP_RFD)
    with pytest.raises(discos.DiscosError, match="unknown step mode"):
        ctx.step(*args, ctx.params(p), 0, mode=2)
    # nothing was launched: the ions are untouched
    assert np.array_equal(host(args[0]), pos)


def test_wet_step_rfd_shifted_kernels_at_tile_edges():
    """Random finite difference with the largest step (delta = 0.1 h): ions just below
    the lower edge of a tile's gathered cells (x, y, z = 14 - eps or 30 - eps on a 32^3
    grid with 16^3 force tiles) reach the tile's first nodes only through their shifted
    kernels; the step must still equal the oracle's."""
    from paper_2204_14167_amd import discos
    w = workloads.WORKLOADS["dirichlet_32x32x32_n256"]
    p = workloads.make_params(w)
    delta = 0.1 * w.h
    p["rfd_delta"] = delta
    pos, q, ids, species = workloads.make_ions(w)
    rng = np.random.default_rng(41)
    n = w.n
    k = np.arange(n)
    edge = np.where(rng.uniform(size=n) < 0.5, 14.0, 30.0) - rng.uniform(1e-4, 0.02, n)
    axis = k % 3
    for d in range(3):
        sel = axis == d
        pos[d, sel] = edge[sel]
    pos[2] = np.clip(pos[2], 1.0, w.nz - 1.0)
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    ctx = _ctx(w)
    dp = ctx.params(p)
    args = (dev(pos), dev(q), dev(ids), dev(species))
    ref, _, _ = dynamics.wet_step(grid, pos, q, species, ids, p, 3, rfd_delta=delta, near="brute")
    ctx.step(*args, dp, 3, mode=discos.STEP_WET | discos.STEP_RFD)
    ctx.check()
    got = by_id(host(args[0]), host(args[2]), ids)
    r = np.linalg.norm(min_image(got - ref, grid.L)) / np.linalg.norm(min_image(ref - pos, grid.L))
    log(f"rfd at tile edges rel={r:.3e}")
    assert r < TOL

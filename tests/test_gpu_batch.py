"""GPU parity of the batched dry step: every channel of a batch advanced in one set of
launches equals the oracle's dry step of that channel alone (relative L2 of the
displacements <= 1e-10), equals a single-channel context, and the captured hipGraph
replays equal the eager launches."""
import numpy as np
import pytest

from oracle import dynamics, electrostatics as es
import workloads
from tests.gpu_util import TOL, by_id, dev, host, log, min_image

pytestmark = pytest.mark.gpu


def _batch(count, seed):
    from paper_2204_14167_amd import discos
    reps, pos, q, ids, species = workloads.make_batch(count, seed=seed)
    for r in reps:
        r["mob_coef"] = workloads.batch_channel_params(r)["mob_coef"]
    p = workloads.batch_channel_params(reps[0])
    b = discos.Batch(reps, 1.0, p)
    return b, reps, pos, q, ids, species


def _channel(b, reps, arrays, r):
    lo, hi = b.offsets[r], b.offsets[r + 1]
    pos, q, ids, sp = arrays
    return pos[:, lo:hi], q[lo:hi], ids[lo:hi], sp[lo:hi]


def _oracle_check(reps, b, before, after, r, step, sample=None, p=None):
    rep = reps[r]
    w = rep["workload"]
    if p is None:
        p = workloads.batch_channel_params(rep)
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    pos0, q0, ids0, sp0 = _channel(b, reps, before, r)
    order = np.argsort(ids0)
    pos0, q0, ids0, sp0 = pos0[:, order], q0[order], ids0[order], sp0[order]
    targets = None
    if sample is not None and w.n > sample:
        targets = np.sort(np.random.default_rng(r).choice(w.n, sample, replace=False))
    ref, _, _ = dynamics.dry_step(grid, pos0, q0, sp0, ids0, p, step, targets=targets)
    pos1, _, ids1, _ = _channel(b, reps, after, r)
    want = ids0 if targets is None else ids0[targets]
    got = by_id(pos1, ids1, want)
    old = pos0 if targets is None else pos0[:, targets]
    err = np.linalg.norm(min_image(got - ref, grid.L)) / np.linalg.norm(min_image(ref - old, grid.L))
    return err


def _host_all(t):
    return tuple(host(x) for x in t)


def test_batch_matches_oracle_per_channel():
    b, reps, pos, q, ids, sp = _batch(12, seed=101)
    log(f"batch of {len(reps)}: " + ", ".join(f"{r['nx']}x{r['ny']}x{r['nz']}/{r['n']}" for r in reps))
    arrays = (dev(pos), dev(q), dev(ids), dev(sp))
    before = _host_all(arrays)
    b.step(*arrays, step=3)
    b.check()
    after = _host_all(arrays)
    for r in range(len(reps)):
        err = _oracle_check(reps, b, before, after, r, 3, sample=400)
        log(f"channel {r} rel {err:.3e}")
        assert err < TOL
    # every channel keeps its own ions, as a permutation of its slots
    for r in range(len(reps)):
        _, _, ids1, _ = _channel(b, reps, after, r)
        assert np.array_equal(np.sort(ids1), np.arange(reps[r]["n"]))


def test_batch_equals_single_contexts():
    from paper_2204_14167_amd import discos
    b, reps, pos, q, ids, sp = _batch(40, seed=202)
    arrays = (dev(pos), dev(q), dev(ids), dev(sp))
    b.step(*arrays, step=7)
    b.check()
    got = _host_all(arrays)
    worst = 0.0
    for r, rep in enumerate(reps):
        w = rep["workload"]
        ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n)
        p = workloads.batch_channel_params(rep)
        lo, hi = b.offsets[r], b.offsets[r + 1]
        one = (dev(pos[:, lo:hi]), dev(q[lo:hi]), dev(ids[lo:hi]), dev(sp[lo:hi]))
        ctx.step(*one, ctx.params(p), 7)
        ctx.check()
        ref_pos, _, ref_ids, _ = _host_all(one)
        gpos, _, gids, _ = _channel(b, reps, got, r)
        a = by_id(gpos, gids, np.arange(w.n))
        c = by_id(ref_pos, ref_ids, np.arange(w.n))
        d0 = min_image(c - pos[:, lo:hi], np.array([w.nx, w.ny, w.nz], float))
        e = np.linalg.norm(min_image(a - c, np.array([w.nx, w.ny, w.nz], float))) / np.linalg.norm(d0)
        worst = max(worst, e)
    log(f"batched vs single contexts: worst rel {worst:.3e}")
    assert worst < 1e-12


def test_graph_replays_match_eager():
    import torch
    b, reps, pos, q, ids, sp = _batch(16, seed=303)
    A = [dev(pos), dev(q), dev(ids), dev(sp)]
    B = [torch.empty_like(t) for t in A]
    for s in range(4):
        for x, y in zip(B, A):
            y_copy = y.clone()
            x.copy_(y_copy)
        torch.cuda.synchronize()
        b.step(*B, step=s, graph=True)      # captured on the first pass, replayed after
        torch.cuda.synchronize()
        b.step(*A, step=s)                  # eager, from the same state
        b.check()
        pa, pb = host(A[0]), host(B[0])
        ia, ib = host(A[2]), host(B[2])
        # the same channels, the same ions: compare per channel by id
        for r in range(len(reps)):
            lo, hi = b.offsets[r], b.offsets[r + 1]
            n = hi - lo
            xa = by_id(pa[:, lo:hi], ia[lo:hi], np.arange(n))
            xb = by_id(pb[:, lo:hi], ib[lo:hi], np.arange(n))
            assert np.abs(xa - xb).max() < 1e-9, (s, r)
        log(f"replay {s} matches eager")


def test_tuning_keeps_results():
    b, reps, pos, q, ids, sp = _batch(24, seed=404)
    arrays = (dev(pos), dev(q), dev(ids), dev(sp))
    before = _host_all(arrays)
    cfg = b.tune(*arrays)
    log(f"tuned: {cfg}")
    assert cfg["spread_tile"] in (8, 16) and cfg["interp_tile"] in (8, 16)
    assert cfg["ion_block"] in (64, 128, 256)
    assert cfg["interp_direct"] in (0, 8, 24, 64, 1 << 30)
    assert cfg["spread_direct"] in (0, 8, 24, 64, 1 << 30)
    assert cfg["bin"] in (2, 4)
    # tuning does not move the ions
    assert np.array_equal(host(arrays[0]), before[0])
    b.step(*arrays, step=1, graph=True)
    b.check()
    after = _host_all(arrays)
    for r in (0, 5, 11, 23):
        assert _oracle_check(reps, b, before, after, r, 1, sample=300) < TOL


def test_batch_rejections():
    from paper_2204_14167_amd import discos
    reps, pos, q, ids, sp = workloads.make_batch(3, seed=5)
    p = workloads.batch_channel_params(reps[0])
    bad = [dict(r) for r in reps]
    bad[1]["nx"] = 24  # not a power of two
    with pytest.raises(discos.DiscosError):
        discos.Batch(bad, 1.0, p)
    bad = [dict(r) for r in reps]
    bad[2]["nz"] = 2
    with pytest.raises(discos.DiscosError):
        discos.Batch(bad, 1.0, p)
    b = discos.Batch(reps, 1.0, p)
    with pytest.raises(discos.DiscosError, match="flags"):
        b._rc(discos.lib().discos_batch_step(b.handle, None, None, None, None, 0, 8, None))


def test_full_512_channel_batch_sampled():
    b, reps, pos, q, ids, sp = _batch(512, seed=None)
    log(f"512 channels, {pos.shape[1]} ions, {sum(r['nx'] * r['ny'] * r['nz'] for r in reps)} cells")
    arrays = (dev(pos), dev(q), dev(ids), dev(sp))
    before = _host_all(arrays)
    b.tune(*arrays)
    b.step(*arrays, step=0, graph=True)
    b.check()
    after = _host_all(arrays)
    for r in np.random.default_rng(9).choice(512, 10, replace=False):
        err = _oracle_check(reps, b, before, after, int(r), 0, sample=150)
        log(f"channel {r} ({reps[r]['nx']}x{reps[r]['ny']}x{reps[r]['nz']}, {reps[r]['n']} ions) rel {err:.3e}")
        assert err < TOL


def _custom_params(rep):
    """Parameters of a custom channel: the shared physics and tables, the channel's noise
    key, and its mobility coefficients (the stored fit of the nearest tabulated height;
    any coefficients are valid inputs for parity)."""
    p = workloads.make_params(rep["workload"], with_tables=False)
    p["p3m_table"], p["p3m_dr"] = workloads.load_p3m_table()
    p["mob_coef"] = rep["mob_coef"]
    p["seed"] = rep["seed"]
    return p


def _custom_batch(shapes, bc_types, bc_values, seed):
    """Batch of channels with the given (nx, ny, nz, n) and walls (all channels share the
    wall types, as a batch requires)."""
    from paper_2204_14167_amd import discos
    rng = np.random.default_rng(seed)
    reps, parts = [], []
    for r, (nx, ny, nz, n) in enumerate(shapes):
        w = workloads.Workload(f"custom_{r}", nx, ny, nz, n, bc_types, bc_values,
                               seed=int(rng.integers(1, 2**62)))
        rep = dict(nx=nx, ny=ny, nz=nz, n=n, bc_values=bc_values, seed=w.seed + 1000, workload=w)
        height = min((16, 32, 64, 128), key=lambda H: abs(H - nz))
        coef = workloads.load_mobility_coef(float(height))
        rep["mob_coef"] = np.stack([coef, coef])
        reps.append(rep)
        parts.append(workloads.make_ions(w))
    pos = np.concatenate([a[0] for a in parts], axis=1)
    q = np.concatenate([a[1] for a in parts])
    ids = np.concatenate([a[2] for a in parts]).astype(np.int32)
    sp = np.concatenate([a[3] for a in parts]).astype(np.int32)
    b = discos.Batch(reps, 1.0, _custom_params(reps[0]))
    return b, reps, pos, q, ids, sp


@pytest.mark.parametrize("walls", [((workloads.NEUMANN, workloads.NEUMANN), (0.0, 0.0)),
                                   ((workloads.DIRICHLET, workloads.NEUMANN), (0.5, 0.0))])
def test_batch_z_solve_paths(walls):
    """Every z-solve path of a batch: segment lengths 8 (nz = 8, 32) and 16 (nz = 37, 64),
    the per-mode Thomas sweep (nz = 160 > 128), and, with both walls Neumann, the singular
    kappa = 0 mode of each channel; against the oracle and against single contexts."""
    from paper_2204_14167_amd import discos
    shapes = [(16, 16, 32, 200), (32, 16, 64, 512), (16, 16, 37, 120), (16, 32, 160, 600),
              (16, 16, 8, 40)]
    b, reps, pos, q, ids, sp = _custom_batch(shapes, walls[0], walls[1], seed=303)
    arrays = (dev(pos), dev(q), dev(ids), dev(sp))
    before = _host_all(arrays)
    b.step(*arrays, step=2)
    b.check()
    after = _host_all(arrays)
    for r in range(len(reps)):
        p = _custom_params(reps[r])
        err = _oracle_check(reps, b, before, after, r, 2, p=p)
        log(f"{walls[0]} channel {shapes[r]} vs oracle rel {err:.3e}")
        assert err < TOL
        w = reps[r]["workload"]
        ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n)
        lo, hi = b.offsets[r], b.offsets[r + 1]
        one = (dev(pos[:, lo:hi]), dev(q[lo:hi]), dev(ids[lo:hi]), dev(sp[lo:hi]))
        ctx.step(*one, ctx.params(p), 2)
        ctx.check()
        ref_pos, _, ref_ids, _ = _host_all(one)
        gpos, _, gids, _ = _channel(b, reps, after, r)
        L = np.array([w.nx, w.ny, w.nz], float)
        a = by_id(gpos, gids, np.arange(w.n))
        c = by_id(ref_pos, ref_ids, np.arange(w.n))
        e = np.linalg.norm(min_image(a - c, L)) / np.linalg.norm(min_image(c - pos[:, lo:hi], L))
        log(f"  vs single context rel {e:.3e}")
        assert e < 1e-12


@pytest.mark.parametrize("walls", [((workloads.DIRICHLET, workloads.DIRICHLET), (1.0, 0.0)),
                                   ((workloads.NEUMANN, workloads.NEUMANN), (0.0, 0.0))])
def test_batch_bin_edges(walls):
    """Cell-list bins of 4 cells (near-field search radius 1 bin for psi = 4 h) and of 2
    cells give the oracle's step on every channel.  The heights leave the last slab 1, 2, 3
    or 4 cells thick, so the image slabs above the upper wall sit off the slab grid by 6,
    4, 2 or 0 cells (two, one or no extra image slabs); widths of 16 cells give 4 bins of
    4 cells, the narrowest that a 3-bin search window allows."""
    from paper_2204_14167_amd import discos
    shapes = [(16, 16, 13, 160), (16, 32, 14, 200), (32, 16, 15, 240), (16, 16, 16, 180),
              (32, 32, 33, 600), (16, 16, 6, 80), (64, 16, 22, 400)]
    b, reps, pos, q, ids, sp = _custom_batch(shapes, walls[0], walls[1], seed=808)
    for bin_cells in (4, 2):
        b.set_bin(bin_cells)
        arrays = (dev(pos), dev(q), dev(ids), dev(sp))
        before = _host_all(arrays)
        b.step(*arrays, step=5)
        b.check()
        after = _host_all(arrays)
        for r in range(len(reps)):
            err = _oracle_check(reps, b, before, after, r, 5, p=_custom_params(reps[r]))
            log(f"bin {bin_cells}, {walls[0]} channel {shapes[r]} vs oracle rel {err:.3e}")
            assert err < TOL
    with pytest.raises(discos.DiscosError, match="2 or 4"):
        b.set_bin(3)

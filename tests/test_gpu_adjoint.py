"""GPU parity of the hand-written adjoint: U, Q and the vector-Jacobian product
(positions, charges, wall fields, applied field) against the oracle's reverse sweep
to relative L2 <= 1e-10; central differences of the GPU forward itself; the
autograd.Function; the 1,048,576-ion, 256x256x128 dielectric case on a sample."""
import numpy as np
import pytest

from oracle import adjoint, electrostatics as es
import workloads
from tests.gpu_util import TOL, dev, host, log, rel_l2

pytestmark = pytest.mark.gpu

D, N = es.DIRICHLET, es.NEUMANN


def _case(bc, nx=16, ny=32, nz=12, n=300, seed=3):
    grid = es.Grid(nx, ny, nz)
    rng = np.random.default_rng(seed)
    pos, q = workloads.random_ions(nx, ny, nz, n, seed)
    pos[2, :n // 8] = rng.uniform(0.0, 2.5, n // 8)
    pos[2, n // 8:n // 4] = nz - rng.uniform(0.0, 2.5, n // 4 - n // 8)
    pos[2, 0], pos[2, 1] = 0.0, float(nz)
    bcv = [rng.normal(scale=0.3, size=(ny, nx)) for _ in range(2)]
    if bc == (N, N):
        shift = (q.sum() + bcv[0].sum() + bcv[1].sum()) / (2 * nx * ny)
        bcv = [b - shift for b in bcv]
    p = dict(eps=1.0 / (4 * np.pi * 4.46), bc_types=bc, bc_values=tuple(bcv),
             e_ext=np.array([0.1, 0.02, -0.03]), eta=1.0 / (6 * np.pi))
    return grid, pos, q, p


def _ctx(grid, n):
    from paper_2204_14167_amd import discos
    return discos.Context(grid.nx, grid.ny, grid.nz, grid.h, max(n, 1))


def _gpu_grads(ctx, pos, q, p, gU, gQ):
    prm = ctx.params(p)
    dpos, dq = dev(pos), dev(q)
    out, phi = ctx.energy_flux(dpos, dq, prm)
    g = dev(np.array([gU, gQ]))
    res = ctx.energy_flux_backward(dpos, dq, prm, phi, g)
    ctx.check()
    return host(out), {k: host(v) for k, v in res.items()}


@pytest.mark.parametrize("bc", [(D, D), (N, N), (D, N), (N, D)])
def test_forward_and_backward_parity(bc):
    grid, pos, q, p = _case(bc)
    log(f"adjoint parity bc={bc}")
    ref = adjoint.gradients(grid, pos, q, p, gU=0.7, gQ=1.3)
    out, got = _gpu_grads(_ctx(grid, pos.shape[1]), pos, q, p, 0.7, 1.3)
    assert abs(out[0] - ref["U"]) <= TOL * abs(ref["U"])
    assert abs(out[1] - ref["Q"]) <= TOL * abs(ref["Q"])
    assert rel_l2(got["pos"], ref["pos"]) < TOL
    assert rel_l2(got["q"], ref["q"]) < TOL
    assert rel_l2(got["bc_lo"], ref["bc"][0]) < TOL
    assert rel_l2(got["bc_hi"], ref["bc"][1]) < TOL
    assert rel_l2(got["e_ext"], ref["e_ext"]) < TOL


@pytest.mark.parametrize("shape", [(8, 16, 9, 120), (64, 8, 20, 700), (32, 32, 37, 900)])
def test_parity_tile_shapes(shape):
    """Grids narrower than a tile (one tile spans the periodic x or y axis), several
    tiles with a ragged last z tile, wall-hugging ions: the face accumulation of the
    transposed E_x gather and the 4^3 gradient windows at tile seams."""
    nx, ny, nz, n = shape
    grid, pos, q, p = _case((N, D), nx=nx, ny=ny, nz=nz, n=n, seed=11)
    ref = adjoint.gradients(grid, pos, q, p, gU=0.4, gQ=-0.9)
    out, got = _gpu_grads(_ctx(grid, pos.shape[1]), pos, q, p, 0.4, -0.9)
    log(f"adjoint shape {shape}: pos {rel_l2(got['pos'], ref['pos']):.2e} "
        f"bc_lo {rel_l2(got['bc_lo'], ref['bc'][0]):.2e}")
    assert abs(out[1] - ref["Q"]) <= TOL * abs(ref["Q"])
    for k in ("pos", "q"):
        assert rel_l2(got[k], ref[k]) < TOL
    assert rel_l2(got["bc_lo"], ref["bc"][0]) < TOL
    assert rel_l2(got["bc_hi"], ref["bc"][1]) < TOL
    assert rel_l2(got["e_ext"], ref["e_ext"]) < TOL


@pytest.mark.parametrize("gU,gQ", [(1.0, 0.0), (0.0, 1.0)])
def test_each_functional_alone(gU, gQ):
    grid, pos, q, p = _case((D, N), seed=5)
    ref = adjoint.gradients(grid, pos, q, p, gU=gU, gQ=gQ)
    _, got = _gpu_grads(_ctx(grid, pos.shape[1]), pos, q, p, gU, gQ)
    for k in ("pos", "q"):
        assert rel_l2(got[k], ref[k]) < TOL
    assert rel_l2(np.stack([got["bc_lo"], got["bc_hi"]]), np.stack(ref["bc"])) < TOL
    if gQ == 0.0:
        assert np.all(got["e_ext"] == 0.0)


def test_backward_reusing_the_forward_cell_list():
    """DISCOS_ADJ_REUSE_CELLS gives the gradients of a rebuilt cell list; after another
    call rebuilt the context's list (or with another n) the backward pass rebuilds it."""
    grid, pos, q, p = _case((D, N))
    n = pos.shape[1]
    ctx = _ctx(grid, n)
    prm = ctx.params(p)
    dpos, dq = dev(pos), dev(q)
    g = dev(np.array([0.7, -1.3]))
    out, phi = ctx.energy_flux(dpos, dq, prm)
    ref = {k: host(v) for k, v in ctx.energy_flux_backward(dpos, dq, prm, phi, g).items()}
    # right after the forward pass
    out, phi = ctx.energy_flux(dpos, dq, prm)
    got = {k: host(v) for k, v in ctx.energy_flux_backward(dpos, dq, prm, phi, g, reuse_cells=True).items()}
    for k in ref:
        assert rel_l2(got[k], ref[k]) < 1e-12, k
    # another call rebuilds the list in between (as many ions, elsewhere, other charges):
    # the flag must not reuse it
    from paper_2204_14167_amd import discos
    other = pos.copy()
    other[0] = np.mod(other[0] + 3.3, grid.L[0])
    ctx.spread(discos.SPREAD_CHARGE, dev(other), dev(q[::-1].copy()), prm)
    got = {k: host(v) for k, v in ctx.energy_flux_backward(dpos, dq, prm, phi, g, reuse_cells=True).items()}
    for k in ref:
        assert rel_l2(got[k], ref[k]) < 1e-12, k
    ctx.check()


def test_no_ions():
    grid, pos, q, p = _case((D, D))
    ref = adjoint.gradients(grid, pos[:, :0], q[:0], p, gU=1.0, gQ=1.0)
    ctx = _ctx(grid, 1)
    prm = ctx.params(p)
    import torch
    empty_pos = torch.zeros((3, 0), dtype=torch.float64, device="cuda")
    empty_q = torch.zeros(0, dtype=torch.float64, device="cuda")
    out, phi = ctx.energy_flux(empty_pos, empty_q, prm)
    res = ctx.energy_flux_backward(empty_pos, empty_q, prm, phi, dev(np.array([1.0, 1.0])))
    ctx.check()
    assert abs(host(out)[0] - ref["U"]) <= TOL * abs(ref["U"]) and host(out)[1] == 0.0
    assert rel_l2(host(res["bc_lo"]), ref["bc"][0]) < TOL
    assert np.all(host(res["e_ext"]) == 0.0)


def test_fd_4096_ions_on_gpu():
    """Central differences (step 1e-6) of the GPU forward along random position
    directions, and parity with the oracle, on the 4,096-ion 32^3 dielectric case."""
    w = workloads.WORKLOADS["dielectric_32x32x32_n4096"]
    P = workloads.make_params(w)
    pos, q, _, _ = workloads.make_ions(w)
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    p = dict(eps=P["eps"], bc_types=P["bc_types"], bc_values=P["bc_values"], e_ext=P["e_ext"],
             eta=P["eta"])
    ctx = _ctx(grid, w.n)
    out, got = _gpu_grads(ctx, pos, q, p, 1.0, 1.0)
    ref = adjoint.gradients(grid, pos, q, p, 1.0, 1.0)
    assert rel_l2(got["pos"], ref["pos"]) < TOL and rel_l2(got["q"], ref["q"]) < TOL
    prm = ctx.params(p)
    rng = np.random.default_rng(2)
    e = 1e-6
    for _ in range(3):
        v = rng.normal(size=pos.shape)
        v /= np.linalg.norm(v)
        fp = host(ctx.energy_flux(dev(pos + e * v), dev(q), prm)[0]).sum()
        fm = host(ctx.energy_flux(dev(pos - e * v), dev(q), prm)[0]).sum()
        fd = (fp - fm) / (2 * e)
        an = float((got["pos"] * v).sum())
        log(f"fd {fd:.12e} adjoint {an:.12e}")
        assert abs(fd - an) < 1e-5 * np.linalg.norm(got["pos"])


def test_autograd_function_matches_backward():
    import torch
    from paper_2204_14167_amd.autograd import energy_flux
    grid, pos, q, p = _case((D, D), seed=6)
    ctx = _ctx(grid, pos.shape[1])
    tp = dev(pos).requires_grad_(True)
    tq = dev(q).requires_grad_(True)
    lo = dev(p["bc_values"][0]).requires_grad_(True)
    hi = dev(p["bc_values"][1]).requires_grad_(True)
    e = torch.tensor(p["e_ext"], dtype=torch.float64, requires_grad=True)
    U, Q = energy_flux(tp, tq, lo, hi, e, ctx, p)
    (0.5 * U + 2.0 * Q).backward()
    ref = adjoint.gradients(grid, pos, q, p, gU=0.5, gQ=2.0)
    assert rel_l2(host(tp.grad), ref["pos"]) < TOL
    assert rel_l2(host(tq.grad), ref["q"]) < TOL
    assert rel_l2(host(lo.grad), ref["bc"][0]) < TOL
    assert rel_l2(host(hi.grad), ref["bc"][1]) < TOL
    assert rel_l2(e.grad.numpy(), ref["e_ext"]) < TOL
    # only Q: no energy term in the gradient
    tq.grad = None
    U, Q = energy_flux(tp, tq, lo, hi, e, ctx, p)
    Q.backward()
    ref = adjoint.gradients(grid, pos, q, p, gU=0.0, gQ=1.0)
    assert rel_l2(host(tq.grad), ref["q"]) < TOL


def test_headline_1m_ions_sampled():
    """The 1,048,576-ion, 256x256x128 dielectric channel with E_x = 0.1: U, Q, the wall
    and field gradients in full, position / charge gradients on a sample."""
    w = workloads.WORKLOADS["dielectric_256x256x128_n1048576"]
    P = workloads.make_params(w)
    pos, q, _, _ = workloads.make_ions(w)
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    p = dict(eps=P["eps"], bc_types=P["bc_types"], bc_values=P["bc_values"], e_ext=P["e_ext"],
             eta=P["eta"])
    log("headline adjoint: GPU")
    out, got = _gpu_grads(_ctx(grid, w.n), pos, q, p, 1.0, 1.0)
    sample = np.arange(0, w.n, 997)
    log("headline adjoint: oracle")
    ref = adjoint.gradients(grid, pos, q, p, 1.0, 1.0, targets=sample)
    log(f"U {out[0]!r} / {ref['U']!r}; Q {out[1]!r} / {ref['Q']!r}")
    assert abs(out[0] - ref["U"]) <= TOL * abs(ref["U"])
    assert abs(out[1] - ref["Q"]) <= TOL * abs(ref["Q"])
    assert rel_l2(got["pos"][:, sample], ref["pos"]) < TOL
    assert rel_l2(got["q"][sample], ref["q"]) < TOL
    assert rel_l2(got["bc_lo"], ref["bc"][0]) < TOL
    assert rel_l2(got["bc_hi"], ref["bc"][1]) < TOL
    assert rel_l2(got["e_ext"], ref["e_ext"]) < TOL

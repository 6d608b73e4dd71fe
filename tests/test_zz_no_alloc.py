"""The no-allocation charge spread (discos_spread_charge_noalloc, a fixed device scratch
array instead of a context) against the context entry point discos_spread on the same
inputs: two calls in a row, the second with a smaller input, on a workload that spans
several tiles and has ions on the walls; wall terms on and off; sizes beyond the fixed
scratch refused before anything runs.  Both paths run the same kernels, so they differ
only by the order of the FP64 atomics: the spread's 1e-13 relative L2 bar."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import dev, host, log, rel_l2

pytestmark = pytest.mark.gpu

EPS = 1.0 / (4.0 * np.pi * 4.46)


def _params(bc, nx, ny, seed):
    rng = np.random.default_rng(seed)
    p = workloads.physical_params()
    p["eps"] = EPS
    p["bc_types"] = bc
    p["bc_values"] = (rng.normal(size=(ny, nx)), rng.normal(size=(ny, nx)))
    return p


def _ions(nx, ny, nz, n, seed):
    pos, q = workloads.random_ions(nx, ny, nz, n, seed, charge="normal")
    pos[2, 0] = 0.0
    pos[2, 1] = float(nz)
    pos[2, 2:n // 4] = np.random.default_rng(seed + 1).uniform(0.0, 2.0, n // 4 - 2)
    return pos, q


def test_noalloc_spread_matches_the_context_spread_twice():
    import torch
    from paper_2204_14167_amd import discos
    cases = [((64, 32, 40), 20000, (0, 1)), ((32, 16, 13), 700, (1, 0))]
    for k, ((nx, ny, nz), n, bc) in enumerate(cases):
        log(f"no-alloc spread call {k}: grid {nx}x{ny}x{nz}, n={n}, walls {bc}")
        pos, q = _ions(nx, ny, nz, n, seed=11 + k)
        p = _params(bc, nx, ny, seed=5 + k)
        ctx = discos.Context(nx, ny, nz, 1.0, n)
        dp = ctx.params(p)
        dpos, dq = dev(pos), dev(q)
        status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
        for add_bc in (False, True):
            op = discos.SPREAD_CHARGE | (discos.SPREAD_ADD_BC if add_bc else 0)
            ref = host(ctx.spread(op, dpos, dq, dp))
            got = host(discos.spread_charge_noalloc((nx, ny, nz, 1.0), dpos, dq, dp,
                                                    add_bc=add_bc, status=status))
            err = rel_l2(got, ref)
            log(f"  add_bc={add_bc}: rel-L2 {err:.2e}")
            assert err < 1e-13
            assert int(host(status)[0]) == discos.OK
        ctx.check()
        ctx.close()


def test_noalloc_spread_flags_and_refusals():
    import torch
    from paper_2204_14167_amd import discos
    nx, ny, nz = 16, 16, 8
    p = discos.Params(_params((0, 0), nx, ny, seed=1), (nx, ny, nz, 1.0))
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    # an ion below the channel is flagged, not read out of bounds
    pos, q = _ions(nx, ny, nz, 50, seed=3)
    pos[2, 7] = -0.5
    log("no-alloc spread: one ion outside the channel")
    discos.spread_charge_noalloc((nx, ny, nz, 1.0), dev(pos), dev(q), p, status=status)
    assert int(host(status)[0]) == discos.E_OUT_OF_DOMAIN
    # the next clean call starts from cleared flags
    pos[2, 7] = 1.0
    discos.spread_charge_noalloc((nx, ny, nz, 1.0), dev(pos), dev(q), p, status=status)
    assert int(host(status)[0]) == discos.OK
    # beyond the fixed scratch: refused on the host
    big = discos.NOALLOC_MAX_IONS + 1
    with pytest.raises(discos.DiscosError) as e:
        discos.spread_charge_noalloc((nx, ny, nz, 1.0), dev(np.zeros((3, big))), dev(np.zeros(big)), p)
    assert e.value.code == discos.E_CAPACITY
    # walls whose type varies per column are not taken
    pm = _params((0, 0), nx, ny, seed=1)
    pm["bc_types"] = (np.zeros((ny, nx), dtype=np.int32), 0)
    with pytest.raises(discos.DiscosError) as e:
        discos.spread_charge_noalloc((nx, ny, nz, 1.0), dev(pos), dev(q),
                                     discos.Params(pm, (nx, ny, nz, 1.0)))
    assert e.value.code == discos.E_ARG
    p2 = discos.Params(_params((0, 0), 1024, 1024, seed=1), (1024, 1024, 8, 1.0))
    with pytest.raises(discos.DiscosError) as e:
        discos.spread_charge_noalloc((1024, 1024, 8, 1.0), dev(pos), dev(q), p2)
    assert e.value.code == discos.E_CAPACITY
    torch.cuda.synchronize()

"""Stage timing of discos_step: every stage, one selected stage (the others read 0),
and reads after recording stopped."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


def test_profile_all_and_selected_stages():
    from paper_2204_14167_amd import discos
    w = workloads.WORKLOADS["dielectric_32x32x32_n4096"]
    p = workloads.make_params(w)
    pos, q, ids, species = workloads.make_ions(w)
    ctx = discos.Context(w.nx, w.ny, w.nz, w.h, w.n)
    dp = ctx.params(p)
    args = (dev(pos), dev(q), dev(ids), dev(species))
    dry = [s for s in ctx.STAGES if s not in ("spread_hy", "stokes", "interp_hy")]
    ctx.profile(True)
    for k in range(3):
        ctx.step(*args, dp, k)
    st = ctx.profile_read()
    assert all(st[s] > 0.0 for s in dry)
    ctx.profile_stages(["near_field", "update"])
    for k in range(3):
        ctx.step(*args, dp, 3 + k)
    st = ctx.profile_read()
    assert st["near_field"] > 0.0 and st["update"] > 0.0
    assert all(st[s] == 0.0 for s in ctx.STAGES if s not in ("near_field", "update"))
    ctx.profile_stages([])
    ctx.step(*args, dp, 6)
    assert all(v == 0.0 for v in ctx.profile_read().values())
    ctx.check()
    assert np.all(np.isfinite(args[0].cpu().numpy()))

"""Pins of the oracle's short-range forces, wall mobility and dry update (CPU only).

  * 9-3 wall potential: force against a central difference of the potential and
    the minimum of Uhat, -xi at y = 3^{1/6} sigma (eq LJ93);
  * LJ: force against a central difference, WCA zero force at its cutoff;
  * fit function: with c3 = c5 = c7 = 0 and the single-wall coefficients it is the
    single-wall mobility of eq singlewall; its derivative against a difference;
    eq mob_analytic tends to 1 mid-way in a wide channel and the stored fits stay
    within their recorded residual of it;
  * dry update: free diffusion statistics (mean 0, variance 2 D dt per axis),
    drift D dt F / kT, reflection at the walls and periodic wrap.
"""
import numpy as np
import pytest

from oracle import dynamics, mobility, shortrange
from oracle.electrostatics import Grid
import workloads


def test_wall_93_force_is_minus_gradient():
    y = np.linspace(0.6, 3.4, 57)
    s, xi, cut = 1.0, 1.3, 3.5
    e = 1e-6
    fd = (shortrange.u93(y + e, s, xi, cut) - shortrange.u93(y - e, s, xi, cut)) / (2 * e)
    np.testing.assert_allclose(shortrange.du93(y, s, xi, cut), fd, rtol=1e-7, atol=1e-8)
    ymin = 3 ** (1 / 6) * s
    assert abs(shortrange.u93_hat(ymin, s, xi) + xi) < 1e-14
    assert shortrange.du93(np.array([ymin]), s, xi, cut)[0] == pytest.approx(0.0, abs=1e-14)
    assert shortrange.u93(np.array([cut]), s, xi, cut)[0] == 0.0
    # both walls push inward; the bottom wall only acts below its cutoff
    Lz = 20.0
    assert shortrange.wall_force(np.array([0.8]), Lz, s, xi, cut)[0] > 0
    assert shortrange.wall_force(np.array([Lz - 0.8]), Lz, s, xi, cut)[0] < 0
    assert shortrange.wall_force(np.array([10.0]), Lz, s, xi, cut)[0] == 0


def test_lj_force_is_minus_gradient():
    r = np.linspace(0.9, 2.4, 31)
    e = 1e-6
    fd = (shortrange.u_lj(r + e, 1.0, 2.0, 2.5) - shortrange.u_lj(r - e, 1.0, 2.0, 2.5)) / (2 * e)
    np.testing.assert_allclose(shortrange.du_lj(r, 1.0, 2.0, 2.5), fd, rtol=1e-7, atol=1e-8)
    wca = 2 ** (1 / 6)
    assert shortrange.du_lj(np.array([wca * (1 - 1e-12)]), 1.0, 1.0, wca)[0] == pytest.approx(0, abs=1e-9)
    L = np.array([10.0, 10.0, 10.0])
    pos = np.array([[1.0, 2.0], [5.0, 5.0], [5.0, 5.0]])
    f = shortrange.lj_pair_forces(L, pos, np.array([0, 0]), np.ones((1, 1)), np.ones((1, 1)), 2.5)
    np.testing.assert_allclose(f[0], [-shortrange.du_lj(np.array([1.0]), 1, 1, 2.5)[0] * -1.0,
                                      shortrange.du_lj(np.array([1.0]), 1, 1, 2.5)[0] * -1.0])


def test_fit_function_reduces_to_single_wall():
    a = 0.8
    y = np.linspace(1.0, 10.0, 50)
    c_par = [1.0, -9 * a / 16, 0.0, 2 * a ** 3 / 16, 0.0, -a ** 5 / 16, 0.0]
    c_perp = [1.0, -9 * a / 8, 0.0, 4 * a ** 3 / 8, 0.0, -a ** 5 / 8, 0.0]
    np.testing.assert_allclose(mobility.gamma_hat(y, c_par),
                               mobility.gamma_single_wall(y, a, mobility.PAR), rtol=1e-14)
    np.testing.assert_allclose(mobility.gamma_hat(y, c_perp),
                               mobility.gamma_single_wall(y, a, mobility.PERP), rtol=1e-14)
    c = [0.9, -0.5, 0.3, -0.08, 0.01, 0.001, 0.03]
    e = 1e-6
    fd = (mobility.gamma_hat(y + e, c) - mobility.gamma_hat(y - e, c)) / (2 * e)
    np.testing.assert_allclose(mobility.dgamma_hat(y, c), fd, rtol=1e-7)


def test_channel_mobility_and_stored_fits():
    for direction in (mobility.PAR, mobility.PERP):
        mid = mobility.gamma_channel(np.array([500.0]), 1.0, 1000.0, direction)[0]
        assert abs(mid - 1.0) < 0.01
        near = mobility.gamma_channel(np.array([1.0]), 1.0, 1000.0, direction)[0]
        single = mobility.gamma_single_wall(np.array([1.0]), 1.0, direction)[0]
        assert abs(1 / near - 1 / single) < 0.01  # the nearest wall dominates
    import json, os
    with open(os.path.join(workloads.DATA_DIR, "mobility_fit.json")) as f:
        fits = json.load(f)
    for key, fit in fits.items():
        Lz = float(key)
        y = np.linspace(0.7, Lz / 2, 100)
        for name, direction in (("parallel", mobility.PAR), ("perpendicular", mobility.PERP)):
            ref = mobility.gamma_channel(y, 1.0, Lz, direction)
            err = np.abs(mobility.gamma_hat(y, fit[name]) - ref).max()
            assert err <= fit[name + "_max_residual"] + 1e-12
            assert err < 0.06


def test_gamma_clamp_and_drift():
    coef = workloads.load_mobility_coef(32)
    z = np.linspace(0.0, 32.0, 1001)
    G = mobility.Gamma(z, 32.0, coef)
    assert G.min() >= 0.0 and G.max() <= 1.0
    dG = mobility.dGamma_perp_dz(z, 32.0, coef)
    e = 1e-6
    zi = z[(z > 1.0) & (z < 15.0)]
    fd = (mobility.Gamma(zi + e, 32.0, coef)[2] - mobility.Gamma(zi - e, 32.0, coef)[2]) / (2 * e)
    np.testing.assert_allclose(mobility.dGamma_perp_dz(zi, 32.0, coef), fd, rtol=1e-6, atol=1e-9)
    # symmetric channel: the drift points away from the nearer wall
    assert np.all(dG[(z > 1.0) & (z < 15.0)] >= 0)
    assert np.all(dG[(z > 17.0) & (z < 31.0)] <= 0)


def _free_params(seed=5):
    p = workloads.physical_params()
    p["mob_coef"] = np.tile(np.array([1.0, 0, 1, 0, 1, 0, 1]), (2, 2, 1))
    p["seed"] = seed
    return p


def test_free_diffusion_statistics():
    grid = Grid(64, 64, 64)
    n = 200_000
    pos = np.full((3, n), 32.0)
    F = np.zeros((3, n))
    species = np.zeros(n, dtype=np.int32)
    ids = np.arange(n)
    p = _free_params()
    disp = dynamics.dry_displacement(grid, pos, F, species, ids, p, step=3)
    D = p["kT"] / (6 * np.pi * p["eta"] * 1.0)
    assert abs(D - 1.0) < 1e-14
    for k in range(3):
        assert abs(disp[k].mean()) < 4 * np.sqrt(2 * D * p["dt"] / n)
        assert abs(disp[k].var() / (2 * D * p["dt"]) - 1.0) < 0.015
    # a constant force adds the deterministic drift D dt F / kT exactly
    F[0] = 3.0
    disp2 = dynamics.dry_displacement(grid, pos, F, species, ids, p, step=3)
    np.testing.assert_allclose(disp2[0] - disp[0], D * p["dt"] * 3.0 / p["kT"], rtol=1e-12)
    np.testing.assert_array_equal(disp2[1:], disp[1:])


def _reflect_by_iteration(z, Lz):
    while z < 0.0 or z > Lz:
        z = -z if z < 0.0 else 2.0 * Lz - z
    return z


def test_reflection_matches_repeated_reflection():
    rng = np.random.default_rng(4)
    Lz = 10.0
    z = np.concatenate([rng.uniform(-95.0, 105.0, 2000), [-10.0, 20.0, -20.0, 30.0, 0.0, 10.0]])
    got = dynamics.reflect_walls(z, Lz)
    ref = np.array([_reflect_by_iteration(v, Lz) for v in z])
    # one crossing is exact; multiple crossings agree to rounding of the fold
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
    one = (z >= -Lz) & (z <= 2 * Lz)
    np.testing.assert_array_equal(got[one], ref[one])
    assert np.all((got >= 0) & (got <= Lz))
    huge = dynamics.reflect_walls(np.array([1e12 + 3.0, -1e12 - 3.0]), Lz)
    assert np.all((huge >= 0) & (huge <= Lz))


def test_reflection_and_wrap():
    z = np.array([-0.5, 10.5, 3.0, -25.0, 0.0, 10.0])
    out = dynamics.reflect_walls(z, 10.0)
    np.testing.assert_allclose(out, [0.5, 9.5, 3.0, 5.0, 0.0, 10.0])
    x = np.array([-0.25, 8.0, 8.25, -8.0, 3.0, -1e-300])
    out = dynamics.wrap_periodic(x, 8.0)
    np.testing.assert_allclose(out, [7.75, 0.0, 0.25, 0.0, 3.0, 0.0])
    assert np.all(out >= 0) and np.all(out < 8.0)


def test_small_dry_step_runs():
    w = workloads.WORKLOADS["dirichlet_32x32x32_n256"]
    p = workloads.make_params(w)
    pos, q, ids, species = workloads.make_ions(w)
    grid = Grid(w.nx, w.ny, w.nz, w.h)
    new, F, parts = dynamics.dry_step(grid, pos, q, species, ids, p, step=0)
    assert np.all(np.isfinite(new))
    assert np.all((new[2] >= 0) & (new[2] <= grid.L[2]))
    assert np.all((new[:2] >= 0) & (new[:2] < grid.L[:2, None]))

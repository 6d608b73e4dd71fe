"""The equilibrium-density check of the stochastic drift (Sec. III, stochastic drift)
has power: free particles under the dry update of eq ions3 (z only, Euler-Maruyama with
reflection, the oracle's mobility fit, 9-3 walls), simulated here in numpy, keep the
Boltzmann profile of the walls with the drift D dGamma_z/dz and pile up where the
mobility is low without it."""
import numpy as np

from oracle import mobility, shortrange
import workloads
from tests.drift_util import profile_deviation, sample_wall_profile, wall_profile_bins

LZ, DT, SIG, XI, CUT = 32.0, 0.01, 1.0, 1.0, 3.5


def _simulate(drift, n=40000, steps=1000, seed=5):
    coef = workloads.load_mobility_coef(LZ)
    rng = np.random.default_rng(seed)
    z = sample_wall_profile(n, LZ, SIG, XI, CUT, rng)
    for _ in range(steps):
        g = mobility.Gamma(z, LZ, coef)[2]
        fz = shortrange.wall_force(z, LZ, SIG, XI, CUT)
        dz = DT * g * fz + rng.standard_normal(n) * np.sqrt(2.0 * g * DT)
        if drift:
            dz += DT * mobility.dGamma_perp_dz(z, LZ, coef)
        z = z + dz
        z = np.where(z < 0.0, -z, z)
        z = np.where(z > LZ, 2.0 * LZ - z, z)
    return z


def test_wall_profile_statistic_accepts_drift_and_flags_its_absence():
    prob = wall_profile_bins(LZ, SIG, XI, CUT)
    on, _ = profile_deviation(_simulate(True), LZ, prob)
    off, ratio = profile_deviation(_simulate(False), LZ, prob)
    assert on < 5.0, on
    assert off > 10.0, (off, ratio)


def test_sampler_matches_profile():
    prob = wall_profile_bins(LZ, SIG, XI, CUT)
    z = sample_wall_profile(100000, LZ, SIG, XI, CUT, np.random.default_rng(3))
    assert profile_deviation(z, LZ, prob)[0] < 5.0
    assert prob[:3].sum() < 1e-12  # the wall keeps ions beyond 0.75 sigma

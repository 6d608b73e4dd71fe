"""The fit tool of the mobility measurement (CPU): its fit function is eq fitfunction
(against the oracle's own implementation), and the bounded least squares recovers a
member of the family exactly and keeps its pole offsets at or above the bound."""
import numpy as np

from oracle import mobility
from paper_2204_14167_amd import mobility_measure as mm


def test_fit_function_is_eq_fitfunction():
    rng = np.random.default_rng(1)
    y = np.linspace(0.0, 12.0, 97)
    for _ in range(5):
        c = rng.normal(size=7)
        c[2::2] = np.abs(c[2::2]) + 0.3
        np.testing.assert_allclose(mm.fit_function(y, c), mobility.gamma_hat(y, c), rtol=1e-13, atol=1e-13)


def test_fit_recovers_a_member_of_the_family():
    c_true = np.array([0.95, -0.5, 0.6, 0.2, 1.5, -0.05, 2.0])
    c_true[0] -= mm.fit_function(np.array([0.0]), c_true)[0]  # passes through (0, 0)
    y = np.linspace(0.125, 12.0, 96)
    c, res = mm.fit(y, mm.fit_function(y, c_true))
    # a seven-parameter rational fit is ill-conditioned: nearby coefficient sets give
    # the same curve, so the recovery is checked on the curve, to 1e-6 of values ~ 1
    assert res < 1e-6
    yy = np.linspace(0.0, 12.0, 1001)
    np.testing.assert_allclose(mm.fit_function(yy, c), mm.fit_function(yy, c_true), atol=1e-5)


def test_fit_keeps_poles_away_from_the_wall():
    # the analytic channel mobility, whose unbounded fit puts poles next to the wall
    y = np.linspace(0.7, 16.0, 200)
    g = mobility.gamma_channel(y, 1.0, 32.0, mobility.PERP)
    c, res = mm.fit(y, g, pole_min=0.25)
    assert min(c[2], c[4], c[6]) >= 0.25 - 1e-12
    f = mm.fit_function(np.linspace(0.0, 16.0, 3201), c)
    assert f.max() < 1.05 and f.min() > -0.1

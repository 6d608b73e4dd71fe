"""Wall-modified dry mobility, written from Sec. II.C and Sec. III.A (test oracle only).

Fit function (eq fitfunction):
    gamma_hat(y) = c1 + c2/(c3 + y) + c4/(c5 + y)^3 + c6/(c7 + y)^5
with y the distance to the nearest wall.  Gamma_k = clamp(gamma_hat_k, 0, 1) for
k in {parallel (x, y), perpendicular (z)}; in a purely dry run Gamma = gamma^tot
(eq diff2 with D^wet = 0).  The paper's fitted constants are not printed, so the
coefficients are inputs.

Analytic channel mobility (eq mob_analytic with eq singlewall), read with the
outer inverse the printed formula lacks and with powers (a/y)^3, (a/y)^5 where
the print shows a/y^3, a/y^5: a sum over wall reflections of single-wall
mobilities, valid for y >~ 0.7 a.
"""
import numpy as np

PAR, PERP = 0, 1


def gamma_hat(y, c):
    c1, c2, c3, c4, c5, c6, c7 = c
    return c1 + c2 / (c3 + y) + c4 / (c5 + y) ** 3 + c6 / (c7 + y) ** 5


def dgamma_hat(y, c):
    c1, c2, c3, c4, c5, c6, c7 = c
    return -c2 / (c3 + y) ** 2 - 3.0 * c4 / (c5 + y) ** 4 - 5.0 * c6 / (c7 + y) ** 6


def gamma_single_wall(y, a, direction):
    """gamma* of eq singlewall for one infinite plane."""
    t = a / np.asarray(y, dtype=np.float64)
    if direction == PAR:
        return 1.0 - 9.0 * t / 16.0 + 2.0 * t ** 3 / 16.0 - t ** 5 / 16.0
    return 1.0 - 9.0 * t / 8.0 + 4.0 * t ** 3 / 8.0 - t ** 5 / 8.0


def gamma_channel(y, a, L, direction, terms=4000):
    """eq mob_analytic (with its outer inverse) for a channel of height L."""
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    acc = np.ones_like(y)
    for n in range(terms):
        sgn = -1.0 if n % 2 else 1.0
        acc += sgn * (1.0 / gamma_single_wall(n * L + y, a, direction) - 1.0)
        acc += sgn * (1.0 / gamma_single_wall((n + 1) * L - y, a, direction) - 1.0)
    return 1.0 / acc


def wall_distance(z, Lz):
    """Distance to the nearest wall and d(distance)/dz (+1 below mid-plane, -1 above)."""
    z = np.asarray(z, dtype=np.float64)
    below = z <= Lz - z
    return np.where(below, z, Lz - z), np.where(below, 1.0, -1.0)


def Gamma(z, Lz, coef):
    """(Gamma_x, Gamma_y, Gamma_z) at heights z; coef [2, 7] = (parallel, perpendicular)."""
    y, _ = wall_distance(z, Lz)
    gp = np.clip(gamma_hat(y, coef[PAR]), 0.0, 1.0)
    gn = np.clip(gamma_hat(y, coef[PERP]), 0.0, 1.0)
    return np.stack([gp, gp, gn])


def dGamma_perp_dz(z, Lz, coef):
    """d Gamma_z / dz (zero where the clamp is active)."""
    y, sgn = wall_distance(z, Lz)
    g = gamma_hat(y, coef[PERP])
    free = (g > 0.0) & (g < 1.0)
    return np.where(free, sgn * dgamma_hat(y, coef[PERP]), 0.0)

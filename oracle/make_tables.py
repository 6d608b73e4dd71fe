"""Offline generator of the two stored input tables (calls only the oracle).

Writes into workloads/data/ (the stored inputs that both sides read):

  p3m_g_peskin4.txt  The free-space grid pair force of the 4-point Peskin kernel
      (the F^P of eq LC, which the paper pre-tabulates as a function of the
      separation).  g(rho) is the mean radial force between two unit charges at
      separation r = rho h through S^es -> Poisson -> J^es, in units of
      1 / (4 pi eps h^2).  Procedure: a triply periodic 64^3 grid, a source
      charge at a random position, the field gathered at rho h along a random
      direction, averaged over placements and directions; the periodic
      neutralising background adds a radial -r / (3 eps V) near the source,
      which is removed.  g(0) = 0 by symmetry.
  mobility_fit.json  Coefficients c1..c7 of eq fitfunction for parallel and
      perpendicular motion in channels of height 16, 32, 64, 128 ion radii.  The
      paper's constants are not printed; following its procedure (a least-squares
      fit that includes the point (0, 0)), the fitted data are the corrected
      eq mob_analytic sampled on y in [0.7 a, Lz / 2].

Run: python -m oracle.make_tables
"""
import json
import os

import numpy as np
from scipy.optimize import least_squares

import workloads

from . import electrostatics as es
from . import mobility

OUT_DIR = workloads.DATA_DIR

RHO_MAX = workloads.P3M_RHO_MAX
DRHO = workloads.P3M_DRHO
N_BOX = workloads.P3M_BOX
PLACEMENTS = workloads.P3M_PLACEMENTS
SEED = workloads.P3M_SEED


def p3m_table():
    grid = es.Grid(N_BOX, N_BOX, N_BOX, 1.0)
    eps = 1.0 / (4.0 * np.pi)
    L = grid.L
    V = float(np.prod(L))
    rho = np.arange(0, int(round(RHO_MAX / DRHO)) + 1) * DRHO
    acc = np.zeros_like(rho)
    # the seeded placements (charge position, directions) are inputs
    srcs, dirs = workloads.p3m_placements()
    for k in range(PLACEMENTS):
        src = srcs[k][:, None]
        dens = es.spread_periodic(grid, src, np.array([1.0]))
        phi = es.periodic_poisson(grid, eps, dens)
        u = dirs[k].copy()
        u /= np.linalg.norm(u, axis=0)
        tgt = np.mod(src + rho[None, :] * u, L[:, None])
        E = es.periodic_grid_field(grid, tgt, phi)
        radial = (E * u).sum(axis=0) + rho / (3.0 * eps * V)
        acc += radial
    g = acc / PLACEMENTS  # F * 4 pi eps h^2 with eps = 1/(4 pi), h = 1
    g[0] = 0.0
    return rho, g


def mobility_fits(heights=(16, 32, 64, 128), a=1.0):
    fits = {}
    for Lz in heights:
        y = np.linspace(0.7 * a, Lz / 2.0, 400)
        out = {}
        for name, direction in (("parallel", mobility.PAR), ("perpendicular", mobility.PERP)):
            target = mobility.gamma_channel(y, a, float(Lz), direction)
            ys = np.concatenate([[0.0], y])
            ts = np.concatenate([[0.0], target])
            x0 = np.array([1.0, -0.6, 0.3, 0.1, 0.05, 0.0, 0.05])

            def resid(c):
                return mobility.gamma_hat(ys, c) - ts

            lo = [-np.inf, -np.inf, 1e-3, -np.inf, 1e-3, -np.inf, 1e-3]
            hi = [np.inf, np.inf, 20.0, np.inf, 20.0, np.inf, 20.0]
            sol = least_squares(resid, x0, bounds=(lo, hi), xtol=1e-15, ftol=1e-15,
                                gtol=1e-15, max_nfev=20000)
            out[name] = [float(v) for v in sol.x]
            out[name + "_max_residual"] = float(np.abs(resid(sol.x)).max())
        fits[str(Lz)] = out
    return fits


def main():
    os.makedirs(OUT_DIR, exist_ok=True)
    rho, g = p3m_table()
    with open(os.path.join(OUT_DIR, "p3m_g_peskin4.txt"), "w") as f:
        f.write("# free-space grid pair force of the 4-point Peskin kernel, "
                "units 1/(4 pi eps h^2)\n")
        f.write(f"# dr={DRHO!r} rho_max={RHO_MAX!r} box={N_BOX} placements={PLACEMENTS} "
                f"seed={SEED}\n")
        for v in g:
            f.write(f"{float(v)!r}\n")
    fits = mobility_fits()
    with open(os.path.join(OUT_DIR, "mobility_fit.json"), "w") as f:
        json.dump(fits, f, indent=1)
    print("g(4) * 16 =", g[int(round(4.0 / DRHO))] * 16.0)
    for k, v in fits.items():
        print(k, v["parallel_max_residual"], v["perpendicular_max_residual"])


if __name__ == "__main__":
    main()

"""The dry DISCOS time step, written from Sec. II.C-II.D (test oracle only).

Stages (Sec. II.D): (1) spread charges, solve Poisson; (2) interpolate the field,
F^P = q E^P, add the P3M near-field correction, the short-range wall force and
the applied field (eq totalforce); (4, dry part) the Euler-Maruyama update of
eq ions3 / eq step2 with the dry diffusion tensor of eq diff1:

  x+_k = x_k + dt D Gamma_k F_k / kT + dt delta_kz D dGamma_z/dz
         + sqrt(2 D Gamma_k dt) W_k,                D = kT / (6 pi eta a)

All terms are evaluated at x^n (Ito).  eq step2 prints the scalar D^dry in the
force and noise terms while eq ions3 uses the tensor D^dry Gamma; the tensor form
is used throughout.  Ions that cross a wall are reflected (z -> -z, or
z -> 2 Lz - z, repeated until inside); x and y are wrapped into [0, L).

Parameters are a plain dict (see the keys read below).
"""
import numpy as np

from . import electrostatics as es
from . import mobility
from . import shortrange
from .rng import TAG_DRY, ion_normals


def total_force(grid, pos, q, species, p, targets=None):
    """F = F^P + sum F^LC + F^W (+ F^R) + q E_ext, eq totalforce; returns (F, parts)."""
    rho, phi, ep, fp = es.grid_force(grid, pos, q, p["eps"], p["bc_types"], p["bc_values"],
                                      p["e_ext"])
    sel = slice(None) if targets is None else targets
    F = fp[:, sel].copy()
    fn = es.near_field(grid, pos, q, p["eps"], p["psi"], p["p3m_table"], p["p3m_dr"],
                       p["bc_types"], targets=targets)
    F += fn
    if p.get("wall_on", True):
        F[2] += shortrange.wall_force(pos[2, sel], grid.L[2], p["wall_sigma"], p["wall_xi"],
                                      p["wall_cut"])
    if p.get("lj_on", False):
        F += shortrange.lj_pair_forces(grid.L, pos, species, p["lj_sigma"], p["lj_xi"],
                                       p["lj_cut_factor"], targets=targets)
    return F, dict(rho=rho, phi=phi, ep=ep, fp=fp, fn=fn)


def wrap_periodic(x, L):
    r = np.fmod(x, L)
    r = np.where(r < 0.0, r + L, r)
    r = np.where(r >= L, r - L, r)
    return np.where(r == 0.0, 0.0, r)


def reflect_walls(z, Lz):
    z = np.array(z, dtype=np.float64)
    if np.any(~np.isfinite(z)):
        raise ValueError("non-finite position")
    while True:
        lo = z < 0.0
        hi = z > Lz
        if not (lo.any() or hi.any()):
            return z
        z = np.where(lo, -z, z)
        z = np.where(hi, 2.0 * Lz - z, z)


def dry_displacement(grid, pos, F, species, ids, p, step):
    """x+ - x^n before reflection / wrapping (eq ions3 dry part, Euler-Maruyama)."""
    kT, dt = p["kT"], p["dt"]
    a = np.asarray(p["radius"])[species]
    D = kT / (6.0 * np.pi * p["eta"] * a)
    Lz = grid.L[2]
    G = np.empty((3, pos.shape[1]))
    dG = np.empty(pos.shape[1])
    coef = np.asarray(p["mob_coef"])
    for s in np.unique(species):
        m = species == s
        G[:, m] = mobility.Gamma(pos[2, m], Lz, coef[s])
        dG[m] = mobility.dGamma_perp_dz(pos[2, m], Lz, coef[s])
    W = ion_normals(p["seed"], step, TAG_DRY, ids)
    disp = dt * D * G * F / kT
    disp[2] += dt * D * dG
    disp += np.sqrt(2.0 * D * G * dt) * W
    return disp


def dry_update(grid, pos, F, species, ids, p, step):
    disp = dry_displacement(grid, pos, F, species, ids, p, step)
    new = pos + disp
    L = grid.L
    new[0] = wrap_periodic(new[0], L[0])
    new[1] = wrap_periodic(new[1], L[1])
    new[2] = reflect_walls(new[2], L[2])
    return new


def dry_step(grid, pos, q, species, ids, p, step):
    """One full dry step; returns (new positions, F, intermediates)."""
    F, parts = total_force(grid, pos, q, species, p)
    new = dry_update(grid, pos, F, species, ids, p, step)
    return new, F, parts

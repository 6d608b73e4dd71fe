"""The DISCOS time step, dry and wet, written from Sec. II.C-II.D (test oracle only).

Stages (Sec. II.D): (1) spread charges, solve Poisson; (2) interpolate the field,
F^P = q E^P, add the P3M near-field correction, the short-range wall force and
the applied field (eq totalforce); (4, dry part) the Euler-Maruyama update of
eq ions3 / eq step2 with the dry diffusion tensor of eq diff1:

  x+_k = x_k + dt D Gamma_k F_k / kT + dt delta_kz D dGamma_z/dz
         + sqrt(2 D Gamma_k dt) W_k,                D = kT / (6 pi eta a)

All terms are evaluated at x^n (Ito).  eq step2 prints the scalar D^dry in the
force and noise terms while eq ions3 uses the tensor D^dry Gamma; the tensor form
is used throughout.  Ions that cross a wall are reflected (z -> -z, or
z -> 2 Lz - z, repeated until inside; the paper uses specular reflection at the
walls in its electro-osmosis runs); x and y are wrapped into [0, L).

Wet step (Sec. II.D stages 3-4, eq disc_stokes_temp, eq step1, eq step2): the
same forces F^n are spread with S^hy, the fluctuating no-slip Stokes problem is
solved once for v^n, and the ions move by the midpoint rule

  x*      = x^n + (dt/2) J(x^n) v^n                     (wrapped / reflected)
  x^{n+1} = x^n + dt J(x*) v^n + [dry terms of eq step2 at x^n]

with the optional thermal forcing f^th = kT div_x S^hy (eq thermforce) by the random
finite difference (kT/delta) [S(x + delta/2 W) W - S(x - delta/2 W) W], one
Gaussian W per ion from its own stream.  The dry terms use the caller's dry radius
(a_d of eq einstein; an infinite radius means no dry diffusion) and the same
Gamma coefficients as the dry step.

Parameters are a plain dict (see the keys read below).
"""
import numpy as np

from . import electrostatics as es
from . import mobility
from . import shortrange
from . import stokes
from .rng import TAG_DRY, TAG_RFD, ion_normals


def total_force(grid, pos, q, species, p, targets=None, near="brute", pot=None):
    """F = F^P + sum F^LC + F^W (+ F^R) + q E_ext, eq totalforce; returns (F, parts).

    The grid part uses all ions; with `targets` the forces (interpolation,
    near-field, short-range) are evaluated for that subset only.  near="pairs"
    takes the near-field sum from the k-d tree pair search, for large systems.
    `pot` = (rho, phi) of es.potential for these ions, if already computed.
    """
    sel = slice(None) if targets is None else np.asarray(targets)
    if pot is None:
        pot = es.potential(grid, pos, q, p["eps"], p["bc_types"], p["bc_values"])
    rho, phi = pot
    ext = es.ghost_extend(grid, p["eps"], p["bc_types"], p["bc_values"], phi)
    ep = es.interp_field(grid, pos[:, sel], *es.face_fields(grid, ext))
    fp = q[sel][None, :] * (ep + np.asarray(p["e_ext"], dtype=np.float64)[:, None])
    F = fp.copy()
    if near == "pairs":
        fn = es.near_field_pairs(grid, pos, q, p["eps"], p["psi"], p["p3m_table"], p["p3m_dr"],
                                 p["bc_types"], targets=targets)
    else:
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
    """Specular reflection at z = 0 and z = Lz, repeated until inside.

    Written in closed form so that arbitrarily large excursions cost O(1): a
    single crossing maps z < 0 to -z and z > Lz to 2 Lz - z exactly; anything
    farther is folded with period 2 Lz (the composition of the reflections).
    """
    z = np.array(z, dtype=np.float64)
    if np.any(~np.isfinite(z)):
        raise ValueError("non-finite position")
    out = z.copy()
    one_lo = (z < 0.0) & (z >= -Lz)
    one_hi = (z > Lz) & (z <= 2.0 * Lz)
    far = (z < -Lz) | (z > 2.0 * Lz)
    out[one_lo] = -z[one_lo]
    out[one_hi] = 2.0 * Lz - z[one_hi]
    t = np.fmod(z[far], 2.0 * Lz)
    t = np.where(t < 0.0, t + 2.0 * Lz, t)
    out[far] = np.where(t <= Lz, t, 2.0 * Lz - t)
    return out


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


def dry_step(grid, pos, q, species, ids, p, step, targets=None, near="brute", pot=None):
    """One full dry step; returns (new positions, F, intermediates).  With
    `targets` only those ions are advanced (all ions still source the fields);
    near="pairs" takes the near-field sum from the pair search; `pot` as in
    total_force."""
    F, parts = total_force(grid, pos, q, species, p, targets=targets, near=near, pot=pot)
    sel = slice(None) if targets is None else np.asarray(targets)
    new = dry_update(grid, pos[:, sel], F, species[sel], ids[sel], p, step)
    return new, F, parts


def confine(grid, pos):
    """x, y wrapped into [0, L), z reflected into [0, Lz]."""
    out = np.empty_like(pos)
    out[0] = wrap_periodic(pos[0], grid.L[0])
    out[1] = wrap_periodic(pos[1], grid.L[1])
    out[2] = reflect_walls(pos[2], grid.L[2])
    return out


def hydro_kernels(p, species):
    """Per-ion hydrodynamic kernels (w, beta) from p["hydro_kernel"] ([nspecies][2], w = 0
    for the 4-point Peskin kernel), or None when every species uses the Peskin kernel."""
    hk = p.get("hydro_kernel")
    if hk is None:
        return None
    hk = np.asarray(hk, dtype=np.float64).reshape(-1, 2)
    if np.all(hk[:, 0] == 0):
        return None
    return hk[np.asarray(species, dtype=np.int64)]


def hydro_walls(p):
    """(lower, upper) slip flags of the hydrodynamic walls, p["slip"] (default no-slip)."""
    sl = p.get("slip", (False, False))
    return bool(sl[0]), bool(sl[1])


def _spread(grid, pos, F, kernels, slack=0.0, slip=(False, False)):
    if kernels is None:
        return stokes.spread_force(grid, pos, F, slack=slack, slip=slip)
    return stokes.spread_force_kernels(grid, pos, F, kernels, slack=slack, slip=slip)


def _interp(grid, pos, u, v, w, kernels, slip=(False, False)):
    if kernels is None:
        return stokes.interp_velocity(grid, pos, u, v, w, slip=slip)
    return stokes.interp_velocity_kernels(grid, pos, u, v, w, kernels, slip=slip)


def thermal_forcing(grid, pos, ids, kT, delta, seed, step, kernels=None, slip=(False, False)):
    """f^th = kT div_x S^hy (eq thermforce) by the random finite difference
    (kT / delta) [S(x + delta/2 W) W - S(x - delta/2 W) W], W ~ N(0, I) per ion."""
    if not delta > 0.0:
        raise ValueError("delta must be positive")
    W = ion_normals(seed, step, TAG_RFD, ids)
    half = 0.5 * delta * W
    if np.abs(half).max(initial=0.0) >= grid.h:
        raise ValueError("random finite difference shift of a cell or more")
    plus = _spread(grid, pos + half, W, kernels, slack=grid.h, slip=slip)
    minus = _spread(grid, pos - half, W, kernels, slack=grid.h, slip=slip)
    return tuple(kT / delta * (a - b) for a, b in zip(plus, minus))


def wet_step(grid, pos, q, species, ids, p, step, noise=True, rfd_delta=0.0, near="brute",
             targets=None):
    """One wet step (eq disc_stokes_temp, eq step1, eq step2); returns
    (new positions of `targets` (all ions by default), F, intermediates)."""
    F, parts = total_force(grid, pos, q, species, p, near=near)
    kern = hydro_kernels(p, species)
    slip = hydro_walls(p)
    fx, fy, fz = _spread(grid, pos, F, kern, slip=slip)
    if rfd_delta > 0.0:
        tx, ty, tz = thermal_forcing(grid, pos, ids, p["kT"], rfd_delta, p["seed"], step, kern,
                                     slip=slip)
        fx, fy, fz = fx + tx, fy + ty, fz + tz
    if noise:
        nfx, nfy, nfz = stokes.noise_force(grid, p["kT"], p["eta"], p["dt"], p["seed"], step,
                                           slip=slip)
        fx, fy, fz = fx + nfx, fy + nfy, fz + nfz
    u, v, w, _ = stokes.solve_stokes(grid, p["eta"], fx, fy, fz, slip=slip)
    sel = slice(None) if targets is None else np.asarray(targets)
    x0 = pos[:, sel]
    dt = p["dt"]
    ksel = None if kern is None else kern[sel]
    V0 = _interp(grid, x0, u, v, w, ksel, slip)
    mid = confine(grid, x0 + 0.5 * dt * V0)
    V1 = _interp(grid, mid, u, v, w, ksel, slip)
    disp = dt * V1 + dry_displacement(grid, x0, F[:, sel], species[sel], ids[sel], p, step)
    new = confine(grid, x0 + disp)
    return new, F, dict(parts, V0=V0, V1=V1, mid=mid, vel=(u, v, w))

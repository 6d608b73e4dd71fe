"""Seeded synthetic inputs shared by the GPU library's tests, the benchmark and
the oracle's tests.  A neutral module: neither the oracle nor the library owns it,
and it imports neither.

This module holds none of the method's arithmetic: it draws ion positions and
charges, names the workloads with their sizes, sets the reduced-unit constants
and reads the two stored input tables (the P3M pair-force table and the wall
mobility fit coefficients).

Reduced units: kT = e = h = 1, ion radius a = h, eps = 1 / (4 pi 4.46) (Bjerrum
length 4.46 a, water at 298 K over a_t = 0.157 nm), eta = 1 / (6 pi) so that the
dry diffusion coefficient kT / (6 pi eta a) is 1, dt = 0.01 (about 1/100 of the
diffusive time a^2 / D, the ratio the paper uses), near-field cutoff psi = 4 h
(the 4-point kernel radius, as in the paper's runs), 9-3 wall with sigma = a,
xi = kT and cutoff 3.5 sigma.
"""
import json
import os
from dataclasses import dataclass, field

import numpy as np

DATA_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")
MASTER_SEED = 220414167

DIRICHLET = 0
NEUMANN = 1


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    n: int
    bc_types: tuple
    bc_values: tuple            # scalar value per wall (phi_b or sigma)
    e_ext: tuple = (0.0, 0.0, 0.0)
    n_plus: int = None          # number of +1 ions (rest are -1); default n/2
    steps: int = 1
    h: float = 1.0
    seed: int = MASTER_SEED
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    # 1:1 electrolyte, grounded walls, one dry step
    "dirichlet_32x32x32_n256": Workload(
        "dirichlet_32x32x32_n256", 32, 32, 32, 256, (DIRICHLET, DIRICHLET), (0.0, 0.0),
        seed=MASTER_SEED + 1),
    # dielectric walls (eps_b/eps = 1/40 -> Neumann limit), applied E_x, 100 dry steps
    "dielectric_128x128x64_n65536": Workload(
        "dielectric_128x128x64_n65536", 128, 128, 64, 65536, (NEUMANN, NEUMANN), (0.0, 0.0),
        e_ext=(0.1, 0.0, 0.0), steps=100, seed=MASTER_SEED + 2),
    # electro-osmosis set-up: charged walls, counter-ion excess, one wet evaluation
    "eo_stokes_128x128x128_n262144": Workload(
        "eo_stokes_128x128x128_n262144", 128, 128, 128, 262144, (NEUMANN, NEUMANN),
        (-0.25, -0.25), e_ext=(0.1, 0.0, 0.0), n_plus=135168, seed=MASTER_SEED + 3),
    # the headline channel: 1 M ions on 256 x 256 x 128, dielectric walls, applied E_x
    "dielectric_256x256x128_n1048576": Workload(
        "dielectric_256x256x128_n1048576", 256, 256, 128, 1048576, (NEUMANN, NEUMANN),
        (0.0, 0.0), e_ext=(0.1, 0.0, 0.0), seed=MASTER_SEED + 5),
    # small sub-case of the headline channel at the same density (finite differences)
    "dielectric_32x32x32_n4096": Workload(
        "dielectric_32x32x32_n4096", 32, 32, 32, 4096, (NEUMANN, NEUMANN), (0.0, 0.0),
        e_ext=(0.1, 0.0, 0.0), seed=MASTER_SEED + 5),
}


def physical_params():
    return dict(kT=1.0, eps=1.0 / (4.0 * np.pi * 4.46), eta=1.0 / (6.0 * np.pi), dt=0.01,
                psi=4.0, wall_on=True, wall_sigma=1.0, wall_xi=1.0, wall_cut=3.5,
                lj_on=False, radius=np.array([1.0, 1.0]))


# Placements that define the grid pair-force table of the P3M correction: a unit charge
# at a uniform position of a periodic box of P3M_BOX^3 unit cells, and normally
# distributed directions (normalised by the table builders) for the separations
# 0, P3M_DRHO, ..., P3M_RHO_MAX cells, P3M_PLACEMENTS times, drawn in that order from one
# seeded stream.
P3M_BOX, P3M_DRHO, P3M_RHO_MAX, P3M_PLACEMENTS, P3M_SEED = 64, 1.0 / 64.0, 6.0, 400, 20414167


def p3m_placements():
    """(src [P, 3] charge positions, dirs [P, 3, nrho] unnormalised directions)."""
    nrho = int(round(P3M_RHO_MAX / P3M_DRHO)) + 1
    rng = np.random.default_rng(P3M_SEED)
    src = np.empty((P3M_PLACEMENTS, 3))
    dirs = np.empty((P3M_PLACEMENTS, 3, nrho))
    for k in range(P3M_PLACEMENTS):
        src[k] = rng.uniform(0.0, float(P3M_BOX), size=(3, 1))[:, 0]
        dirs[k] = rng.normal(size=(3, nrho))
    return src, dirs


def load_p3m_table():
    """(g, dr): tabulated free-space grid pair force of the 4-point Peskin kernel,
    g(i dr) for rho = r / h, written by the oracle's table tool."""
    path = os.path.join(DATA_DIR, "p3m_g_peskin4.txt")
    dr = None
    vals = []
    with open(path) as f:
        for line in f:
            if line.startswith("#"):
                if "dr=" in line:
                    dr = float(line.split("dr=")[1].split()[0])
                continue
            vals.append(float(line))
    return np.array(vals), dr


def load_mobility_coef(lz_over_a):
    """[2, 7] fit coefficients (parallel, perpendicular) for a channel of height
    lz_over_a ion radii, written by the oracle's table tool."""
    with open(os.path.join(DATA_DIR, "mobility_fit.json")) as f:
        fits = json.load(f)
    key = str(int(round(lz_over_a)))
    if key not in fits:
        raise KeyError(f"no mobility fit for Lz/a = {key}; available: {sorted(fits)}")
    return np.array([fits[key]["parallel"], fits[key]["perpendicular"]])


def make_params(w: Workload, with_tables=True):
    """Parameter dict for workload w (same keys on both sides)."""
    p = physical_params()
    p["bc_types"] = tuple(w.bc_types)
    p["bc_values"] = tuple(np.full((w.ny, w.nx), float(v)) for v in w.bc_values)
    p["e_ext"] = np.array(w.e_ext, dtype=np.float64)
    p["seed"] = w.seed + 1000
    if with_tables:
        p["p3m_table"], p["p3m_dr"] = load_p3m_table()
        coef = load_mobility_coef(w.nz * w.h / 1.0)
        p["mob_coef"] = np.stack([coef, coef])
    return p


def make_ions(w: Workload, seed=None):
    """Positions [3, n] (x, y uniform in the box, z uniform in [a, Lz - a]),
    charges (+1 for the first n_plus ions, -1 for the rest), ids and species
    (0 for cations, 1 for anions)."""
    rng = np.random.default_rng(w.seed if seed is None else seed)
    a = 1.0
    L = np.array([w.nx, w.ny, w.nz], dtype=np.float64) * w.h
    pos = np.empty((3, w.n))
    pos[0] = rng.uniform(0.0, L[0], w.n)
    pos[1] = rng.uniform(0.0, L[1], w.n)
    pos[2] = rng.uniform(a, L[2] - a, w.n)
    n_plus = w.n // 2 if w.n_plus is None else w.n_plus
    q = np.where(np.arange(w.n) < n_plus, 1.0, -1.0)
    ids = np.arange(w.n, dtype=np.int32)
    species = np.where(q > 0, 0, 1).astype(np.int32)
    return pos, q, ids, species


def random_ions(nx, ny, nz, n, seed, h=1.0, zmin=0.0, zmax=None, charge="pm"):
    """Free-form seeded ions for tests: z uniform in [zmin, zmax]."""
    rng = np.random.default_rng(seed)
    L = np.array([nx, ny, nz], dtype=np.float64) * h
    zmax = L[2] if zmax is None else zmax
    pos = np.empty((3, n))
    pos[0] = rng.uniform(0.0, L[0], n)
    pos[1] = rng.uniform(0.0, L[1], n)
    pos[2] = rng.uniform(zmin, zmax, n)
    if charge == "pm":
        q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    else:
        q = rng.normal(size=n)
    return pos, q


def make_batch(count=512, seed=None):
    """Independent channels for the batched step: nx, ny drawn from {16, 32, 64}, nz
    from {32, 64}, ion counts log-uniform on [64, 4096] (even: half +1, half -1), a
    grounded top wall and a bottom wall potential uniform in [-2, 2] kT/e, one noise
    key per channel.  Returns (channels, pos [3, N], q, ids, species) with the ions of
    channel r at entries off_r .. off_r + n_r - 1 and ids 0 .. n_r - 1 per channel."""
    rng = np.random.default_rng(MASTER_SEED + 4 if seed is None else seed)
    reps, parts = [], []
    for r in range(count):
        nx = int(rng.choice([16, 32, 64]))
        ny = int(rng.choice([16, 32, 64]))
        nz = int(rng.choice([32, 64]))
        n = int(round(np.exp(rng.uniform(np.log(64.0), np.log(4096.0)))))
        n -= n % 2
        phi_lo = float(rng.uniform(-2.0, 2.0))
        w = Workload(f"channel_{r}", nx, ny, nz, n, (DIRICHLET, DIRICHLET), (phi_lo, 0.0),
                     seed=int(rng.integers(1, 2**62)))
        pos, q, ids, species = make_ions(w)
        reps.append(dict(nx=nx, ny=ny, nz=nz, n=n, bc_values=(phi_lo, 0.0), seed=w.seed + 1000,
                         workload=w))
        parts.append((pos, q, ids, species))
    pos = np.concatenate([a[0] for a in parts], axis=1) if parts else np.zeros((3, 0))
    q = np.concatenate([a[1] for a in parts])
    ids = np.concatenate([a[2] for a in parts]).astype(np.int32)
    species = np.concatenate([a[3] for a in parts]).astype(np.int32)
    return reps, pos, q, ids, species


def batch_channel_params(rep):
    """Parameter dict of one channel of a batch (the same keys as make_params)."""
    w = rep["workload"]
    p = make_params(w)
    p["seed"] = rep["seed"]
    return p


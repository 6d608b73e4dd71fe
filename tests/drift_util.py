"""Equilibrium-density statistic of the stochastic-drift check (Sec. III, stochastic
drift): free particles in the channel are uniform in z at equilibrium whatever their
mobility, so a wrong or missing stochastic drift shows as a density excess or deficit
near the walls, where the mobility varies fastest."""
import numpy as np


def z_edges(Lz):
    """Bins of width h/4 .. h next to each wall, coarse bins in the middle."""
    near = np.array([0.0, 0.25, 0.5, 0.75, 1.0, 1.5, 2.0, 3.0, 4.0])
    mid = np.linspace(4.0, Lz - 4.0, 5)[1:-1]
    return np.unique(np.concatenate([near, mid, Lz - near[::-1]]))


def density_deviation(z, Lz):
    """Largest |count - expected| / sigma over the z bins (binomial sigma of uniform
    positions) and the ratio count / expected per bin."""
    edges = z_edges(Lz)
    n = z.size
    counts, _ = np.histogram(z, edges)
    p = np.diff(edges) / Lz
    expect = n * p
    sigma = np.sqrt(n * p * (1.0 - p))
    return float(np.abs((counts - expect) / sigma).max()), counts / expect


def wall_profile_bins(Lz, sigma, xi, cut, fine=20000):
    """Probability of each bin of z_edges(Lz) under the Boltzmann density
    exp(-(U(z) + U(Lz - z)) / kT), kT = 1, of the 9-3 wall potential U (midpoint rule on
    a fine grid)."""
    from oracle import shortrange
    edges = z_edges(Lz)
    z = (np.arange(fine) + 0.5) * (Lz / fine)
    u = shortrange.u93(z, sigma, xi, cut) + shortrange.u93(Lz - z, sigma, xi, cut)
    w = np.exp(-u)
    mass, _ = np.histogram(z, edges, weights=w)
    return mass / mass.sum()


def sample_wall_profile(n, Lz, sigma, xi, cut, rng):
    """z drawn from the Boltzmann density of the two walls by rejection."""
    from oracle import shortrange
    out = np.empty(0)
    while out.size < n:
        z = rng.uniform(0.0, Lz, 2 * n)
        u = shortrange.u93(z, sigma, xi, cut) + shortrange.u93(Lz - z, sigma, xi, cut)
        umin = -2.0 * xi  # each wall's potential is bounded below by -xi (shifted at the cut)
        keep = rng.uniform(size=z.size) < np.exp(-(u - umin))
        out = np.concatenate([out, z[keep]])
    return out[:n]


def profile_deviation(z, Lz, prob):
    """Largest |count - expected| / sigma over the bins of z_edges(Lz) for bin
    probabilities prob, and count / expected per bin (bins of zero mass skipped)."""
    n = z.size
    counts, _ = np.histogram(z, z_edges(Lz))
    expect = n * prob
    ok = expect > 0.5
    sigma = np.sqrt(n * prob * (1.0 - prob))
    dev = np.zeros_like(expect)
    dev[ok] = (counts[ok] - expect[ok]) / sigma[ok]
    ratio = np.where(ok, counts / np.maximum(expect, 1e-300), 1.0)
    return float(np.abs(dev).max()), ratio

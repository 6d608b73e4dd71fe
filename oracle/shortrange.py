"""Short-range forces, written from Sec. II.B.2 of the paper (test oracle only).

Wall potential: the 9-3 form of eq LJ93, Uhat(y) = (3^{3/2}/2) xi [(s/y)^9 - (s/y)^3],
shifted to zero at the cutoff y_c as in eq potential, and zero for y >= y_c
(the printed zero branch reads "y_c >= y", taken as y >= y_c).  y is the distance
to a wall: z for the bottom wall and Lz - z for the top wall, so
F_z = -U'(z) + U'(Lz - z).

Ion-ion pair force (eq potential / eq closerange): shifted 12-6 Lennard-Jones,
WCA when the cutoff is 2^{1/6} sigma.
"""
import numpy as np

C93 = 1.5 * np.sqrt(3.0)  # 3^{3/2} / 2


def u93_hat(y, sigma, xi):
    return C93 * xi * ((sigma / y) ** 9 - (sigma / y) ** 3)


def u93(y, sigma, xi, cut):
    """Shifted, truncated 9-3 wall potential."""
    y = np.asarray(y, dtype=np.float64)
    inside = (y > 0.0) & (y < cut)
    ys = np.where(inside, y, cut)
    return np.where(inside, u93_hat(ys, sigma, xi) - u93_hat(cut, sigma, xi), 0.0)


def du93(y, sigma, xi, cut):
    """dU/dy of the shifted 9-3 potential (zero outside 0 < y < cut)."""
    y = np.asarray(y, dtype=np.float64)
    inside = (y > 0.0) & (y < cut)
    ys = np.where(inside, y, cut)
    d = C93 * xi * (-9.0 * sigma ** 9 / ys ** 10 + 3.0 * sigma ** 3 / ys ** 4)
    return np.where(inside, d, 0.0)


def wall_force(z, Lz, sigma, xi, cut):
    """z-component of the force from both walls on ions at heights z."""
    z = np.asarray(z, dtype=np.float64)
    return -du93(z, sigma, xi, cut) + du93(Lz - z, sigma, xi, cut)


def u_lj(r, sigma, xi, cut):
    r = np.asarray(r, dtype=np.float64)
    inside = (r > 0.0) & (r < cut)
    rs = np.where(inside, r, cut)
    hat = lambda x: 4.0 * xi * ((sigma / x) ** 12 - (sigma / x) ** 6)
    return np.where(inside, hat(rs) - hat(cut), 0.0)


def du_lj(r, sigma, xi, cut):
    r = np.asarray(r, dtype=np.float64)
    inside = (r > 0.0) & (r < cut)
    rs = np.where(inside, r, cut)
    d = 4.0 * xi * (-12.0 * sigma ** 12 / rs ** 13 + 6.0 * sigma ** 6 / rs ** 7)
    return np.where(inside, d, 0.0)


def lj_pair_forces(L, pos, species, sigma_mat, xi_mat, cut_factor, targets=None):
    """sum_j F^R_ij = -rhat_ij dU/dr with per-pair (sigma_ij, xi_ij) and cutoff
    cut_factor * sigma_ij; minimum image in x and y; brute force."""
    n = pos.shape[1]
    targets = np.arange(n) if targets is None else np.asarray(targets)
    out = np.zeros((3, len(targets)))
    for t, i in enumerate(targets):
        d = pos[:, i:i + 1] - pos
        d[0] -= L[0] * np.round(d[0] / L[0])
        d[1] -= L[1] * np.round(d[1] / L[1])
        r = np.sqrt((d * d).sum(axis=0))
        sig = sigma_mat[species[i], species]
        xi = xi_mat[species[i], species]
        mask = (np.arange(n) != i) & (r < cut_factor * sig)
        rr = np.where(mask, r, 1.0)
        du = np.where(mask, du_lj(rr, sig, xi, cut_factor * sig), 0.0)
        out[:, t] = (-du / rr * d).sum(axis=1)
    return out

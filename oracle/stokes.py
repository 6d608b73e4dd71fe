"""Overdamped Stokes with no-slip or slip walls on the MAC grid, written from Sec. II.A
(eq stokes, eq disc_stokes, eq fluidbc, eq kernel1 / kernel2, the image construction of
Fig. folded and the ghost rule for interpolation).

Part of the test oracle (test infrastructure only).

Layout (staggered / MAC): u on x-faces (i h, (j+1/2) h, (k+1/2) h) as [nz][ny][nx],
v on y-faces, w on z-faces ((i+1/2) h, (j+1/2) h, k h) as [nz+1][ny][nx] with
k = 0 and nz on the walls, pressure at cell centres [nz][ny][nx].  Every wall has
w = 0 on its face.  At a no-slip wall the tangential components have ghosts
u_{-1} = -u_0 (zero at the wall, second order); at a slip wall (zero tangential stress,
eq fluidbc) u_{-1} = +u_0; mirrored at the top.  `slip` = (lower, upper) selects the
type of each wall (default no-slip).

Discrete operator (eq disc_stokes):   G p - eta lap_h v = f,   D v = 0
  (G_x p)_i = (p_i - p_{i-1}) / h on x-faces, likewise y; (G_z p)_k = (p_k - p_{k-1}) / h
  on interior z-faces; (D v) = sum of face differences / h; lap_h the 7-point
  Laplacian on each face grid with the ghost rules above.

Stochastic stress (eq disc_stokes_temp): f_noise = sqrt(2 kT eta / (dV dt)) div_h Z,
with Z symmetric, diagonal entries at cell centres of variance 2, off-diagonal
entries on cell edges of variance 1; the xz and yz edges that lie on a no-slip wall
have variance 2 and those on a slip wall variance 0 (a slip wall carries no
tangential stress), the readings under which the discrete fluctuation-dissipation
balance holds exactly with these ghost rules (pinned by the covariance identity in
the tests).

Two slip walls leave the kappa = 0 tangential problem singular (constant flow is free
and a net force has no steady solution).  Like the kappa = 0 mode of a periodic box,
that mode is solved with its z-mean force removed and its z-mean velocity zero.  The paper puts Delta t under the square root and also calls the Gaussian
"scaled by 1/sqrt(dt)"; it is counted once.
"""
import numpy as np
from scipy.linalg import solve_banded

from . import esc
from .peskin import node_weights
from .rng import TAG_STRESS_DIAG, TAG_STRESS_EDGE, normal_pair


def _check(grid, pos, slack=0.0):
    if grid.nz < 4:
        raise ValueError("nz must be >= 4")
    if (np.any(~np.isfinite(pos)) or np.any(pos[2] < -slack)
            or np.any(pos[2] > grid.L[2] + slack)):
        raise ValueError("ion outside the channel")


def _tsign(slip):
    """Image sign of the tangential components at the (lower, upper) wall."""
    return (1.0 if slip[0] else -1.0), (1.0 if slip[1] else -1.0)


def spread_force(grid, pos, F, slack=0.0, slip=(False, False)):
    """S^hy F on the faces with wall images (eq kernel2, Fig. folded).

    The normal component's image is opposite (zero normal mobility at any wall); the
    tangential components' image is opposite at a no-slip wall and equal at a slip
    wall.  x and y components live at cell-centre heights: a node below the wall
    (k < 0) lands on -1-k with the tangential sign.  The z component lives on
    z-faces: a node at k < 0 lands on -k with sign -1, so the wall face itself
    collects f - f = 0; likewise at the top.

    `slack` admits kernel centres up to that far outside the walls (the shifted
    positions of the random finite difference); the same folds apply.
    """
    _check(grid, pos, slack)
    nx, ny, nz, h = grid.nx, grid.ny, grid.nz, grid.h
    out = []
    for comp, offs in ((0, (0.0, 0.5, 0.5)), (1, (0.5, 0.0, 0.5)), (2, (0.5, 0.5, 0.0))):
        ix, wx = node_weights(pos[0], h, offs[0], nx)
        iy, wy = node_weights(pos[1], h, offs[1], ny)
        iz, wz = node_weights(pos[2], h, offs[2])
        s = np.ones_like(wz)
        if comp < 2:
            lo, hi = iz < 0, iz >= nz
            iz = np.where(lo, -1 - iz, np.where(hi, 2 * nz - 1 - iz, iz))
            arr = np.zeros((nz, ny, nx))
            s_lo, s_hi = _tsign(slip)
        else:
            lo, hi = iz < 0, iz > nz
            iz = np.where(lo, -iz, np.where(hi, 2 * nz - iz, iz))
            arr = np.zeros((nz + 1, ny, nx))
            s_lo, s_hi = -1.0, -1.0
        s[lo] = s_lo
        s[hi] = s_hi
        for c in range(5):
            for b in range(5):
                for a in range(5):
                    np.add.at(arr, (iz[:, c], iy[:, b], ix[:, a]),
                              F[comp] * s[:, c] * wx[:, a] * wy[:, b] * wz[:, c] / h ** 3)
        if comp == 2:
            arr[0] = 0.0
            arr[nz] = 0.0
        out.append(arr)
    return tuple(out)


def _kernel_groups(kernels, n):
    """(kernel, ion indices) for each distinct hydrodynamic kernel; kernels is an [n, 2]
    array of (w, beta) per ion (w = 0: 4-point Peskin)."""
    kk = np.asarray(kernels, dtype=np.float64).reshape(n, 2)
    groups = {}
    for i in range(n):
        groups.setdefault((int(kk[i, 0]), float(kk[i, 1])), []).append(i)
    return [(k, np.array(v, dtype=np.int64)) for k, v in groups.items()]


def spread_force_kernels(grid, pos, F, kernels, slack=0.0, slip=(False, False)):
    """S^hy F as spread_force, each ion with its own kernel (oracle.esc): the kernel's
    nodes on the nine-node window, the same wall folds."""
    _check(grid, pos, slack)
    nx, ny, nz, h = grid.nx, grid.ny, grid.nz, grid.h
    out = [np.zeros((nz, ny, nx)), np.zeros((nz, ny, nx)), np.zeros((nz + 1, ny, nx))]
    for kern, idx in _kernel_groups(kernels, pos.shape[1]):
        p = pos[:, idx]
        for comp, offs in ((0, (0.0, 0.5, 0.5)), (1, (0.5, 0.0, 0.5)), (2, (0.5, 0.5, 0.0))):
            ix, wx = esc.node_weights_kernel(p[0], h, offs[0], kern, nx)
            iy, wy = esc.node_weights_kernel(p[1], h, offs[1], kern, ny)
            iz, wz = esc.node_weights_kernel(p[2], h, offs[2], kern)
            s = np.ones_like(wz)
            if comp < 2:
                lo, hi = iz < 0, iz >= nz
                iz = np.where(lo, -1 - iz, np.where(hi, 2 * nz - 1 - iz, iz))
                s_lo, s_hi = _tsign(slip)
            else:
                lo, hi = iz < 0, iz > nz
                iz = np.where(lo, -iz, np.where(hi, 2 * nz - iz, iz))
                s_lo, s_hi = -1.0, -1.0
            s[lo] = s_lo
            s[hi] = s_hi
            f = F[comp, idx]
            for c in range(9):
                for b in range(9):
                    for a in range(9):
                        np.add.at(out[comp], (iz[:, c], iy[:, b], ix[:, a]),
                                  f * s[:, c] * wx[:, a] * wy[:, b] * wz[:, c] / h ** 3)
    out[2][0] = 0.0
    out[2][nz] = 0.0
    return tuple(out)


def interp_velocity_kernels(grid, pos, u, v, w, kernels, slip=(False, False)):
    """J^hy v as interp_velocity, each ion with its own kernel, ghosts five layers deep."""
    _check(grid, pos)
    nx, ny, h = grid.nx, grid.ny, grid.h
    depth = 5
    fields = (_ghost_tangential(u, depth, slip), _ghost_tangential(v, depth, slip),
              _ghost_normal(w, depth))
    out = np.zeros((3, pos.shape[1]))
    for kern, idx in _kernel_groups(kernels, pos.shape[1]):
        p = pos[:, idx]
        for comp, offs in ((0, (0.0, 0.5, 0.5)), (1, (0.5, 0.0, 0.5)), (2, (0.5, 0.5, 0.0))):
            ix, wx = esc.node_weights_kernel(p[0], h, offs[0], kern, nx)
            iy, wy = esc.node_weights_kernel(p[1], h, offs[1], kern, ny)
            iz, wz = esc.node_weights_kernel(p[2], h, offs[2], kern)
            iz = iz + depth
            f = fields[comp]
            acc = np.zeros(idx.size)
            for c in range(9):
                for b in range(9):
                    for a in range(9):
                        acc += wx[:, a] * wy[:, b] * wz[:, c] * f[iz[:, c], iy[:, b], ix[:, a]]
            out[comp, idx] = acc
    return out


def _ghost_tangential(a, depth=3, slip=(False, False)):
    """[nz + 2 depth] cell-height layers with u_{-1-m} = s_lo u_m and
    u_{nz+m} = s_hi u_{nz-1-m}: s = -1 at a no-slip wall, +1 at a slip wall."""
    nz = a.shape[0]
    s_lo, s_hi = _tsign(slip)
    out = np.empty((nz + 2 * depth,) + a.shape[1:])
    out[depth:depth + nz] = a
    for m in range(depth):
        out[depth - 1 - m] = s_lo * a[m]
        out[depth + nz + m] = s_hi * a[nz - 1 - m]
    return out


def _ghost_normal(wf, depth=3):
    """[nz + 1 + 2 depth] face layers with w_{-k} = -w_k and w_{nz+k} = -w_{nz-k}."""
    nz = wf.shape[0] - 1
    out = np.empty((nz + 1 + 2 * depth,) + wf.shape[1:])
    out[depth:depth + nz + 1] = wf
    for k in range(1, depth + 1):
        out[depth - k] = -wf[k]
        out[depth + nz + k] = -wf[nz - k]
    return out


def interp_velocity(grid, pos, u, v, w, slip=(False, False)):
    """J^hy v = dV sum delta(x_i - r) v(r) per component (eq kernel1), ghosts filled
    with the wall rules so the adjoint identity holds with spread_force."""
    _check(grid, pos)
    nx, ny, h = grid.nx, grid.ny, grid.h
    depth = 3
    fields = (_ghost_tangential(u, depth, slip), _ghost_tangential(v, depth, slip),
              _ghost_normal(w, depth))
    out = np.zeros((3, pos.shape[1]))
    for comp, offs in ((0, (0.0, 0.5, 0.5)), (1, (0.5, 0.0, 0.5)), (2, (0.5, 0.5, 0.0))):
        ix, wx = node_weights(pos[0], h, offs[0], nx)
        iy, wy = node_weights(pos[1], h, offs[1], ny)
        iz, wz = node_weights(pos[2], h, offs[2])
        iz = iz + depth
        f = fields[comp]
        for c in range(5):
            for b in range(5):
                for a in range(5):
                    out[comp] += wx[:, a] * wy[:, b] * wz[:, c] * f[iz[:, c], iy[:, b], ix[:, a]]
    return out


# ---- operator -------------------------------------------------------------------

def _lap_tangential(a, h, slip=(False, False)):
    g = _ghost_tangential(a, 1, slip)
    lz = (g[2:] - 2 * a + g[:-2]) / h ** 2
    lx = (np.roll(a, -1, 2) - 2 * a + np.roll(a, 1, 2)) / h ** 2
    ly = (np.roll(a, -1, 1) - 2 * a + np.roll(a, 1, 1)) / h ** 2
    return lx + ly + lz


def _lap_normal(wf, h):
    """Laplacian of w on the interior faces 1..nz-1 (w_0 = w_nz = 0)."""
    lz = (wf[2:] - 2 * wf[1:-1] + wf[:-2]) / h ** 2
    inner = wf[1:-1]
    lx = (np.roll(inner, -1, 2) - 2 * inner + np.roll(inner, 1, 2)) / h ** 2
    ly = (np.roll(inner, -1, 1) - 2 * inner + np.roll(inner, 1, 1)) / h ** 2
    return lx + ly + lz


def apply_stokes(grid, eta, u, v, w, p, slip=(False, False)):
    """(G p - eta lap_h v, D v): force on the faces (w rows on interior faces only)
    and the divergence in the cells.  The plain definition of eq disc_stokes."""
    h = grid.h
    wf = w.copy()
    wf[0] = 0.0
    wf[-1] = 0.0
    fx = (p - np.roll(p, 1, 2)) / h - eta * _lap_tangential(u, h, slip)
    fy = (p - np.roll(p, 1, 1)) / h - eta * _lap_tangential(v, h, slip)
    fz = np.zeros_like(w)
    fz[1:-1] = (p[1:] - p[:-1]) / h - eta * _lap_normal(wf, h)
    div = ((np.roll(u, -1, 2) - u) + (np.roll(v, -1, 1) - v) + (wf[1:] - wf[:-1])) / h
    return fx, fy, fz, div


# ---- solve ----------------------------------------------------------------------

def solve_stokes(grid, eta, fx, fy, fz, slip=(False, False)):
    """Solve eq disc_stokes for (u, v, w, p) with the walls of `slip`; pressure gauge
    mean 0 (and, with two slip walls, the kappa = 0 tangential flow of zero mean for
    the force with its mean removed).

    In-plane DFT; for each mode a banded system in z with unknowns ordered
    (u_k, v_k, w_k, p_k), solved by LU with partial pivoting (LAPACK gbsv).  The
    kappa = 0 mode has a constant-pressure null space and is solved densely with
    the gauge sum_k p_k = 0 replacing the redundant continuity row.  The paper
    solves the same discrete system with preconditioned GMRES.
    """
    nx, ny, nz, h = grid.nx, grid.ny, grid.nz, grid.h
    Fx = np.fft.fft2(fx, axes=(1, 2))
    Fy = np.fft.fft2(fy, axes=(1, 2))
    Fz = np.fft.fft2(fz, axes=(1, 2))
    U = np.zeros_like(Fx)
    V = np.zeros_like(Fy)
    W = np.zeros_like(Fz)
    Pp = np.zeros_like(Fx)
    nu = 4 * nz
    bw = 4
    ih2 = 1.0 / h ** 2
    k = np.arange(nz)
    iu, iv, iw, ip = 4 * k, 4 * k + 1, 4 * k + 2, 4 * k + 3
    # ghost term of the wall rows: u_{-1} = -u_0 adds +1/h^2, u_{-1} = +u_0 adds -1/h^2
    s_lo, s_hi = _tsign(slip)
    wall_extra = np.zeros(nz)
    wall_extra[0] += -s_lo * ih2
    wall_extra[nz - 1] += -s_hi * ih2
    for n_ in range(ny):
        for m in range(nx):
            tx = 2 * np.pi * m / nx
            ty = 2 * np.pi * n_ / ny
            gx = (1 - np.exp(-1j * tx)) / h     # (p_i - p_{i-1}) / h
            gy = (1 - np.exp(-1j * ty)) / h
            dx = (np.exp(1j * tx) - 1) / h      # (u_{i+1} - u_i) / h
            dy = (np.exp(1j * ty) - 1) / h
            k2 = abs(gx) ** 2 + abs(gy) ** 2
            A = {}

            def put(rows, cols, vals):
                for r, c, v_ in zip(np.atleast_1d(rows), np.atleast_1d(cols),
                                    np.broadcast_to(vals, np.shape(np.atleast_1d(rows)))):
                    A[(int(r), int(c))] = v_

            # tangential momentum rows (wall ghosts of `slip`)
            for rows, g in ((iu, gx), (iv, gy)):
                put(rows, rows, eta * (2 * ih2 + k2 + wall_extra))
                put(rows[1:], rows[:-1], -eta * ih2)
                put(rows[:-1], rows[1:], -eta * ih2)
                put(rows, ip, g)
            # normal momentum rows on interior faces; the wall face row is w_0 = 0
            put(iw[:1], iw[:1], 1.0)
            put(iw[1:], iw[1:], eta * (2 * ih2 + k2))
            put(iw[1:], iw[:-1], -eta * ih2)
            put(iw[1:-1], iw[2:], -eta * ih2)
            put(iw[1:], ip[1:], 1.0 / h)
            put(iw[1:], ip[:-1], -1.0 / h)
            # continuity rows
            put(ip, iu, dx)
            put(ip, iv, dy)
            put(ip, iw, -1.0 / h)
            put(ip[:-1], iw[1:], 1.0 / h)
            rhs = np.zeros(nu, dtype=complex)
            rhs[iu] = Fx[:nz, n_, m]
            rhs[iv] = Fy[:nz, n_, m]
            rhs[iw[1:]] = Fz[1:nz, n_, m]
            if m == 0 and n_ == 0:
                # constant pressure is in the null space: the last continuity row
                # (redundant here) becomes the gauge sum_k p_k = 0
                D = np.zeros((nu, nu), dtype=complex)
                for (r, c), v_ in A.items():
                    D[r, c] = v_
                D[nu - 1, :] = 0.0
                D[nu - 1, ip] = 1.0
                rhs[nu - 1] = 0.0
                if slip[0] and slip[1]:
                    # the tangential rows sum to zero: remove the mean force and let
                    # the last row of each component fix the mean flow to zero
                    for rows in (iu, iv):
                        rhs[rows] -= rhs[rows].mean()
                        D[rows[-1], :] = 0.0
                        D[rows[-1], rows] = 1.0
                        rhs[rows[-1]] = 0.0
                x = np.linalg.solve(D, rhs)
            else:
                ab = np.zeros((2 * bw + 1, nu), dtype=complex)
                for (r, c), v_ in A.items():
                    ab[bw + r - c, c] = v_
                x = solve_banded((bw, bw), ab, rhs)
            U[:, n_, m] = x[iu]
            V[:, n_, m] = x[iv]
            W[:nz, n_, m] = x[iw]
            Pp[:, n_, m] = x[ip]
    u = np.real(np.fft.ifft2(U, axes=(1, 2)))
    v = np.real(np.fft.ifft2(V, axes=(1, 2)))
    w = np.real(np.fft.ifft2(W, axes=(1, 2)))
    p = np.real(np.fft.ifft2(Pp, axes=(1, 2)))
    w[0] = 0.0
    w[nz] = 0.0
    return u, v, w, p


# ---- stochastic stress ----------------------------------------------------------

def stress_normals(grid, seed, step):
    """Unit normals of the stress components: (Wxx, Wyy, Wzz) per cell, Wxy per
    cell-height edge, (Wxz, Wyz) per z-level edge (nz + 1 levels).

    Counters: diagonal tag with the cell index (pair 0 -> xx, yy; pair 1 -> zz);
    edge tag with the z-level index ((k ny + j) nx + i, k = 0..nz)
    (pair 0 -> xz, yz; pair 1 -> xy, the latter used for k < nz only).
    """
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    cells = np.arange(nz * ny * nx)
    a, b = normal_pair(seed, step, TAG_STRESS_DIAG, 0, cells)
    c, _ = normal_pair(seed, step, TAG_STRESS_DIAG, 1, cells)
    lev = np.arange((nz + 1) * ny * nx)
    e1, e2 = normal_pair(seed, step, TAG_STRESS_EDGE, 0, lev)
    e3, _ = normal_pair(seed, step, TAG_STRESS_EDGE, 1, lev)
    sh = (nz, ny, nx)
    shl = (nz + 1, ny, nx)
    return (a.reshape(sh), b.reshape(sh), c.reshape(sh), e3.reshape(shl)[:nz],
            e1.reshape(shl), e2.reshape(shl))


def stress_divergence(grid, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz, slip=(False, False)):
    """div_h Z on the faces for the symmetric stress built from unit normals.

    Z_aa = sqrt(2) W_aa at cell centres; Z_xy = W_xy on edges (i h, j h, (k+1/2) h);
    Z_xz = W_xz on edges (i h, (j+1/2) h, k h), Z_yz = W_yz on ((i+1/2) h, j h, k h),
    k = 0..nz, times sqrt(2) on a no-slip wall level (k = 0 or nz) and 0 on a slip one.
    """
    h = grid.h
    nz = grid.nz
    s2 = np.sqrt(2.0)
    Zxx, Zyy, Zzz = s2 * Wxx, s2 * Wyy, s2 * Wzz
    wall = np.ones((nz + 1, 1, 1))
    wall[0] = 0.0 if slip[0] else s2
    wall[-1] = 0.0 if slip[1] else s2
    Zxz = Wxz * wall
    Zyz = Wyz * wall
    Zxy = Wxy
    # x-face (i, j+1/2, k+1/2): d/dx Zxx (cells i-1, i), d/dy Zxy (edges j, j+1), d/dz Zxz (levels k, k+1)
    fx = ((Zxx - np.roll(Zxx, 1, 2)) + (np.roll(Zxy, -1, 1) - Zxy) + (Zxz[1:] - Zxz[:-1])) / h
    # y-face ((i+1/2), j, k+1/2): d/dx Zxy (edges i, i+1), d/dy Zyy (cells j-1, j), d/dz Zyz
    fy = ((np.roll(Zxy, -1, 2) - Zxy) + (Zyy - np.roll(Zyy, 1, 1)) + (Zyz[1:] - Zyz[:-1])) / h
    # z-face (i+1/2, j+1/2, k), interior k = 1..nz-1: d/dx Zxz (edges i, i+1), d/dy Zyz, d/dz Zzz
    fz = np.zeros((nz + 1,) + Wxx.shape[1:])
    fz[1:-1] = ((np.roll(Zxz[1:-1], -1, 2) - Zxz[1:-1]) + (np.roll(Zyz[1:-1], -1, 1) - Zyz[1:-1])
                + (Zzz[1:] - Zzz[:-1])) / h
    return fx, fy, fz


def noise_force(grid, kT, eta, dt, seed, step, slip=(False, False)):
    """sqrt(2 kT eta / (dV dt)) div_h Z (eq disc_stokes_temp)."""
    amp = np.sqrt(2.0 * kT * eta / (grid.dV * dt))
    fx, fy, fz = stress_divergence(grid, *stress_normals(grid, seed, step), slip=slip)
    return amp * fx, amp * fy, amp * fz


def velocity_at_ions(grid, pos, F, eta, kT=0.0, dt=1.0, seed=0, step=0, kernels=None,
                     slip=(False, False)):
    """V = J^hy L^-1 (S^hy F + noise) (eq ions2 without the thermal drift); kernels:
    per-ion hydrodynamic kernels (w, beta), or None for the 4-point Peskin kernel."""
    if kernels is None:
        fx, fy, fz = spread_force(grid, pos, F, slip=slip)
    else:
        fx, fy, fz = spread_force_kernels(grid, pos, F, kernels, slip=slip)
    if kT > 0.0:
        nx_, ny_, nz_ = noise_force(grid, kT, eta, dt, seed, step, slip=slip)
        fx, fy, fz = fx + nx_, fy + ny_, fz + nz_
    u, v, w, p = solve_stokes(grid, eta, fx, fy, fz, slip=slip)
    if kernels is None:
        return interp_velocity(grid, pos, u, v, w, slip=slip), (u, v, w, p)
    return interp_velocity_kernels(grid, pos, u, v, w, kernels, slip=slip), (u, v, w, p)

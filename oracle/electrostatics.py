"""Electrostatics of the slit channel, written from Sec. II.B.1 of the paper.

Part of the test oracle (test infrastructure only): plain FP64 numpy, no
blocking or fusion beyond what the definitions state.

Layout and conventions (the paper is silent on them; they are the readings used
by both implementations):
  * grid (nx, ny, nz, h); box [0, nx h) x [0, ny h) x [0, nz h]; walls at z = 0
    ("lo", index 0) and z = Lz ("hi", index 1).
  * scalar fields (rho, phi) live at cell centres ((i+1/2) h, (j+1/2) h, (k+1/2) h),
    stored as arrays [nz, ny, nx].
  * E_x lives on x-faces (i h, (j+1/2) h, (k+1/2) h), E_y on y-faces, E_z on
    z-faces ((i+1/2) h, (j+1/2) h, k h), k = 0 .. nz (k = 0 and nz on the walls).
  * wall BC types: DIRICHLET (fixed potential phi_b, eq esbc1) or NEUMANN
    (dielectric wall with surface charge sigma in the eps >> eps_b limit,
    eq esbc3).  Gauss's law fixes the sign of the Neumann condition:
    -eps dphi/dz(0+) = sigma_lo and +eps dphi/dz(Lz-) = sigma_hi, the only sign
    for which an all-Neumann system is solvable exactly when it is neutral
    (Sec. II.B.1, closing remark on electro-neutrality).
  * a wall's type is one type for the whole wall, or a map [ny, nx] giving the
    type of each wall column (i, j) (a metal strip on a dielectric wall,
    Sec. IV.B; the closing remark of Sec. II.B.1 lets the wall data vary along
    the wall).  Every rule below then applies column by column: the image sign of
    a folded kernel node is that of its column, the wall term and the ghost
    values of a column follow its type, and the image of a charge takes the type
    of the wall column directly below (above) it.
"""
import numpy as np

from .peskin import node_weights

DIRICHLET = 0
NEUMANN = 1


class Grid:
    def __init__(self, nx, ny, nz, h=1.0):
        self.nx, self.ny, self.nz, self.h = int(nx), int(ny), int(nz), float(h)

    @property
    def L(self):
        return np.array([self.nx * self.h, self.ny * self.h, self.nz * self.h])

    @property
    def dV(self):
        return self.h ** 3


def image_sign(bc):
    """Sign of the image charge (Sec. II.B.1): opposite at a fixed-potential
    wall, like-signed at a dielectric (Neumann) wall; per column for a type map."""
    a = np.asarray(bc)
    if a.ndim == 0:
        return -1.0 if int(a) == DIRICHLET else 1.0
    return np.where(a == DIRICHLET, -1.0, 1.0)


def type_field(grid, bc):
    """[ny, nx] types of a wall's columns (one type broadcast, or the map itself)."""
    a = np.asarray(bc)
    if a.ndim == 0:
        return np.full((grid.ny, grid.nx), int(a))
    if a.shape != (grid.ny, grid.nx):
        raise ValueError("a wall type map must be [ny, nx]")
    return a.astype(np.int64)


def uniform_type(bc):
    """The wall's single type, or None when its columns differ."""
    a = np.unique(np.asarray(bc))
    return int(a[0]) if len(a) == 1 else None


def ion_columns(grid, pos):
    """Wall column (i, j) of each ion: the cell column containing (x, y)."""
    L = grid.L
    ci = np.minimum(np.floor(np.mod(pos[0], L[0]) / grid.h).astype(np.int64), grid.nx - 1)
    cj = np.minimum(np.floor(np.mod(pos[1], L[1]) / grid.h).astype(np.int64), grid.ny - 1)
    return ci, cj


def source_image_signs(grid, pos, bc):
    """Image sign of each ion's image at one wall: the type of its wall column."""
    s = image_sign(bc)
    if np.ndim(s) == 0:
        return np.full(pos.shape[1], s)
    ci, cj = ion_columns(grid, pos)
    return s[cj, ci]


def _check_positions(grid, pos):
    if grid.nz < 4:
        raise ValueError("nz must be >= 4 so a kernel never reaches both walls")
    z = pos[2]
    if np.any(~np.isfinite(pos)) or np.any(z < 0.0) or np.any(z > grid.L[2]):
        raise ValueError("ion outside the channel 0 <= z <= Lz")


def _bc_field(grid, value):
    v = np.zeros((grid.ny, grid.nx)) if value is None else np.asarray(value, dtype=np.float64)
    return np.broadcast_to(v, (grid.ny, grid.nx))


def spread_scalar(grid, pos, w, signs):
    """S applied to per-ion weights w with image folding at the walls.

    Nodes are the cell centres.  A kernel node below the bottom wall (k < 0)
    is the node of the image particle at -z; it lands on cell -1-k with weight
    sign signs[0]; above the top wall (k >= nz) it lands on 2 nz - 1 - k with
    signs[1] (Sec. II.A image construction, Fig. folded; Sec. II.B.1 for the
    charge images).  Result has units of w per volume (kernel of eq kernel2).
    """
    _check_positions(grid, pos)
    nx, ny, nz, h = grid.nx, grid.ny, grid.nz, grid.h
    ix, wx = node_weights(pos[0], h, 0.5, nx)
    iy, wy = node_weights(pos[1], h, 0.5, ny)
    iz, wz = node_weights(pos[2], h, 0.5)
    lo = iz < 0
    hi = iz >= nz
    iz = np.where(lo, -1 - iz, np.where(hi, 2 * nz - 1 - iz, iz))
    s_lo = np.broadcast_to(np.asarray(signs[0], dtype=np.float64), (ny, nx))
    s_hi = np.broadcast_to(np.asarray(signs[1], dtype=np.float64), (ny, nx))
    out = np.zeros((nz, ny, nx))
    w = np.asarray(w, dtype=np.float64)
    for c in range(5):
        for b in range(5):
            for a in range(5):
                # the folded node's sign is that of its own wall column
                col = (iy[:, b], ix[:, a])
                s = np.where(lo[:, c], s_lo[col], np.where(hi[:, c], s_hi[col], 1.0))
                np.add.at(out, (iz[:, c], iy[:, b], ix[:, a]),
                          w * s * wx[:, a] * wy[:, b] * wz[:, c] / h ** 3)
    return out


def spread_charge(grid, pos, q, bc_types):
    """rho = S^es q (eq delta_funcs regularised by the kernel, Sec. II.B.1)."""
    return spread_scalar(grid, pos, q, (image_sign(bc_types[0]), image_sign(bc_types[1])))


def bc_rhs(grid, eps, bc_types, bc_values):
    """Right-hand-side contribution of inhomogeneous wall conditions.

    With the wall between ghost cell -1 and cell 0, a Dirichlet value phi_b
    gives phi_{-1} = 2 phi_b - phi_0 and moves 2 eps phi_b / h^2 to the RHS of
    layer 0; a Neumann wall with -eps dphi/dz = sigma gives
    phi_{-1} = phi_0 + h sigma / eps and moves sigma / h.  Mirror statements
    hold at the top wall for layer nz - 1.
    """
    h = grid.h
    b = np.zeros((grid.nz, grid.ny, grid.nx))
    for wall, layer in ((0, 0), (1, grid.nz - 1)):
        v = _bc_field(grid, bc_values[wall])
        t = type_field(grid, bc_types[wall])
        b[layer] += np.where(t == DIRICHLET, 2.0 * eps * v / h ** 2, v / h)
    return b


def _thomas(lower, diag, upper, rhs):
    """Tridiagonal solve along axis 0, vectorised over the remaining axes."""
    n = rhs.shape[0]
    cp = np.empty(diag.shape, dtype=np.float64)
    dp = np.empty(rhs.shape, dtype=rhs.dtype)
    cp[0] = upper / diag[0]
    dp[0] = rhs[0] / diag[0]
    for k in range(1, n):
        m = diag[k] - lower * cp[k - 1]
        cp[k] = upper / m
        dp[k] = (rhs[k] - lower * dp[k - 1]) / m
    x = np.empty_like(dp)
    x[-1] = dp[-1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


NEUTRALITY_TOL = 1e-10


def solve_poisson(grid, eps, bc_types, rhs, project=False):
    """Solve -eps lap_h phi = rhs (eq poisson) with homogeneous wall ghosts.

    lap_h is the 7-point Laplacian; the ghost rules are phi_{-1} = -phi_0 at a
    Dirichlet wall and phi_{-1} = +phi_0 at a Neumann wall (inhomogeneous parts
    are already in rhs, see bc_rhs).  Route: DFT in x and y, then for each
    in-plane mode a tridiagonal system in z with
    kappa^2 = (4/h^2)(sin^2(pi m/nx) + sin^2(pi n/ny)).  The paper solves the
    same discrete system with geometric multigrid (Sec. II.D stage 1).

    When both walls are Neumann the kappa = 0 system is singular; it is solvable
    only if the system is neutral (Sec. II.B.1).  That mode is solved in the
    least-squares minimum-norm sense, which fixes mean(phi) = 0; a violation of
    neutrality beyond NEUTRALITY_TOL (relative to the sum over layers of the
    absolute plane sums) raises ValueError.  project=True skips that check and
    applies the pseudo-inverse to any rhs (the component along the null space is
    dropped): the adjoint of the minimum-norm solve, used by the gradient sweeps.
    """
    u_lo, u_hi = uniform_type(bc_types[0]), uniform_type(bc_types[1])
    if u_lo is None or u_hi is None:
        return _solve_poisson_mixed(grid, eps, bc_types, rhs)
    bc_types = (u_lo, u_hi)
    nx, ny, nz, h = grid.nx, grid.ny, grid.nz, grid.h
    R = np.fft.fft2(rhs, axes=(1, 2)) * (h * h / eps)
    m = np.arange(nx)
    n = np.arange(ny)
    k2h2 = 4.0 * (np.sin(np.pi * m / nx)[None, :] ** 2 + np.sin(np.pi * n / ny)[:, None] ** 2)
    s_lo = image_sign(bc_types[0])
    s_hi = image_sign(bc_types[1])
    diag = np.broadcast_to(2.0 + k2h2, (nz, ny, nx)).copy()
    diag[0] -= s_lo
    diag[-1] -= s_hi
    singular = bc_types[0] == NEUMANN and bc_types[1] == NEUMANN
    r0 = None
    if singular:
        r0 = R[:, 0, 0].copy()
        total = abs(r0.sum())
        scale = np.abs(r0).sum()
        if not project and total > NEUTRALITY_TOL * max(scale, 1e-300):
            raise ValueError("all-Neumann system is not electro-neutral")
        diag[:, 0, 0] = 1.0 + 2.0  # placeholder, that mode is replaced below
    X = _thomas(-1.0, diag, -1.0, R)
    if singular:
        A0 = (np.diag(np.full(nz, 2.0)) - np.diag(np.ones(nz - 1), 1) - np.diag(np.ones(nz - 1), -1))
        A0[0, 0] = 1.0
        A0[-1, -1] = 1.0
        X[:, 0, 0] = np.linalg.lstsq(A0, r0, rcond=None)[0]
    return np.real(np.fft.ifft2(X, axes=(1, 2)))


def poisson_matrix(grid, eps, bc_types):
    """-eps lap_h with the homogeneous ghost rule of each wall column as a sparse
    matrix on the cells, index (k ny + j) nx + i: 7-point stencil, periodic in x
    and y; the ghost below cell (i, j, 0) is s phi(i, j, 0) with s = -1 for a
    Dirichlet column and +1 for a Neumann one (likewise above layer nz - 1)."""
    from scipy import sparse
    nx, ny, nz, h = grid.nx, grid.ny, grid.nz, grid.h
    c = eps / h ** 2
    idx = np.arange(nz * ny * nx).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []

    def add(r, q, v):
        rows.append(r.ravel())
        cols.append(q.ravel())
        vals.append(np.broadcast_to(v, r.shape).ravel())

    diag = np.full((nz, ny, nx), 6.0 * c)
    diag[0] -= c * image_sign(type_field(grid, bc_types[0]))
    diag[-1] -= c * image_sign(type_field(grid, bc_types[1]))
    add(idx, idx, diag)
    add(idx, np.roll(idx, 1, axis=2), -c)
    add(idx, np.roll(idx, -1, axis=2), -c)
    add(idx, np.roll(idx, 1, axis=1), -c)
    add(idx, np.roll(idx, -1, axis=1), -c)
    add(idx[1:], idx[:-1], -c)
    add(idx[:-1], idx[1:], -c)
    n = nz * ny * nx
    return sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(n, n))


def _solve_poisson_mixed(grid, eps, bc_types, rhs):
    """Exact solve of the mixed-wall problem: a wall whose columns differ couples the
    in-plane Fourier modes, so the matrix of poisson_matrix is factored directly
    (sparse LU).  Such a wall has a Dirichlet column, so the system is nonsingular."""
    from scipy.sparse.linalg import spsolve
    A = poisson_matrix(grid, eps, bc_types).tocsc()
    return spsolve(A, rhs.ravel()).reshape(rhs.shape)


def ghost_extend(grid, eps, bc_types, bc_values, phi, depth=3):
    """phi with `depth` ghost layers below and above, filled from the wall BC.

    Ghost -1-m (m >= 0): Dirichlet 2 phi_b - phi_m, Neumann phi_m + (2m+1) h sigma/eps;
    ghost nz+m: Dirichlet 2 phi_b - phi_{nz-1-m}, Neumann phi_{nz-1-m} + (2m+1) h sigma/eps.
    These reflections are exact for any potential that is affine in z and
    satisfies the BC (Sec. II.B.1: ghosts filled so the BC on phi holds).
    Returned array has shape [nz + 2 depth, ny, nx]; cell k is at index k + depth.
    """
    nz, h = grid.nz, grid.h
    if depth > nz:
        raise ValueError("ghost depth exceeds nz")
    out = np.empty((nz + 2 * depth,) + phi.shape[1:])
    out[depth:depth + nz] = phi
    for m in range(depth):
        for wall in (0, 1):
            v = _bc_field(grid, bc_values[wall])
            t = type_field(grid, bc_types[wall])
            src = phi[m] if wall == 0 else phi[nz - 1 - m]
            dst = depth - 1 - m if wall == 0 else depth + nz + m
            out[dst] = np.where(t == DIRICHLET, 2.0 * v - src, src + (2 * m + 1) * h * v / eps)
    return out


def face_fields(grid, phi_ext, depth=3):
    """E = -grad_h phi on the faces of the extended grid.

    Ex[e, j, i] = -(phi[e, j, i] - phi[e, j, i-1]) / h at x = i h (periodic);
    Ey likewise along y; Ez[e] with e = f + depth is the field on the z-face
    f (z = f h), -(phi[f] - phi[f-1]) / h; index 0 of Ez is unused (nan).
    """
    h = grid.h
    ex = -(phi_ext - np.roll(phi_ext, 1, axis=2)) / h
    ey = -(phi_ext - np.roll(phi_ext, 1, axis=1)) / h
    ez = np.full_like(phi_ext, np.nan)
    ez[1:] = -(phi_ext[1:] - phi_ext[:-1]) / h
    return ex, ey, ez


def _gather(grid, pos, field_ext, offsets, depth):
    """Delta V * sum_n delta(x_i - r_n) f_n over the node set with the given offsets
    (eq kernel1 with the kernel of eq pkernel); z index taken in the extended array."""
    nx, ny, h = grid.nx, grid.ny, grid.h
    ix, wx = node_weights(pos[0], h, offsets[0], nx)
    iy, wy = node_weights(pos[1], h, offsets[1], ny)
    iz, wz = node_weights(pos[2], h, offsets[2])
    iz = iz + depth
    if iz.size and (iz.min() < 0 or iz.max() >= field_ext.shape[0]):
        raise ValueError("interpolation stencil leaves the ghost-extended grid")
    out = np.zeros(pos.shape[1])
    for c in range(5):
        for b in range(5):
            for a in range(5):
                vals = field_ext[iz[:, c], iy[:, b], ix[:, a]]
                w = wx[:, a] * wy[:, b] * wz[:, c]
                out += np.where(w != 0.0, w * np.nan_to_num(vals), 0.0)
    return out


def interp_field(grid, pos, ex, ey, ez, depth=3):
    """E^P = J^es E: each component gathered from its own face set."""
    _check_positions(grid, pos)
    return np.stack([
        _gather(grid, pos, ex, (0.0, 0.5, 0.5), depth),
        _gather(grid, pos, ey, (0.5, 0.0, 0.5), depth),
        _gather(grid, pos, ez, (0.5, 0.5, 0.0), depth),
    ])


def interp_scalar(grid, pos, phi_ext, depth=3):
    """J applied to a cell-centred scalar (ghost-extended)."""
    _check_positions(grid, pos)
    return _gather(grid, pos, phi_ext, (0.5, 0.5, 0.5), depth)


def potential(grid, pos, q, eps, bc_types, bc_values):
    """phi solving eq poisson for the spread charges plus the wall conditions."""
    rho = spread_charge(grid, pos, q, bc_types)
    rhs = rho + bc_rhs(grid, eps, bc_types, bc_values)
    return rho, solve_poisson(grid, eps, bc_types, rhs)


def grid_field_at_ions(grid, pos, q, eps, bc_types, bc_values):
    """E^P of eq efieldop: J^es(-grad_h (-eps lap_h)^-1 S^es q), walls included."""
    rho, phi = potential(grid, pos, q, eps, bc_types, bc_values)
    ext = ghost_extend(grid, eps, bc_types, bc_values, phi)
    ex, ey, ez = face_fields(grid, ext)
    return rho, phi, interp_field(grid, pos, ex, ey, ez)


def grid_force(grid, pos, q, eps, bc_types, bc_values, e_ext=(0.0, 0.0, 0.0)):
    """F^P_i = q_i (E^P_i + E_ext) (Sec. II.B.1; the applied field is an
    external force term of eq totalforce, not a wall condition)."""
    rho, phi, ep = grid_field_at_ions(grid, pos, q, eps, bc_types, bc_values)
    return rho, phi, ep, q[None, :] * (ep + np.asarray(e_ext, dtype=np.float64)[:, None])


def table_lookup(table, dr, rho):
    """Linear interpolation of g at rho = r/h on the uniform table g(i dr)."""
    t = rho / dr
    i = np.floor(t).astype(np.int64)
    f = t - i
    i = np.minimum(i, len(table) - 2)
    return table[i] * (1.0 - f) + table[i + 1] * f


def near_field(grid, pos, q, eps, psi, table, dr, bc_types, targets=None):
    """P3M short-range correction with wall images (eqs coulomb, fullElectro, LC).

    F_i += sum_{j != i, r_ij < psi} (q_i q_j / (4 pi eps)) [1/r^2 - g(r/h)/h^2] rhat_ij
    where g is the tabulated free-space grid pair force (dimensionless,
    F^P = q_i q_j g(r/h) / (4 pi eps h^2)).  Separations use the minimum image
    in x and y.  Each ion j (including j = i) also has an image at
    (x_j, y_j, -z_j) with charge s_lo q_j and at (x_j, y_j, 2 Lz - z_j) with
    charge s_hi q_j; every image within psi of ion i adds the same correction
    (force on i only).  Pairs at zero separation are skipped.  Brute force over
    all pairs.  `targets` restricts the output to a subset of ions (all ions are
    still sources).
    """
    L = grid.L
    h = grid.h
    n = pos.shape[1]
    targets = np.arange(n) if targets is None else np.asarray(targets)
    s = (source_image_signs(grid, pos, bc_types[0]), source_image_signs(grid, pos, bc_types[1]))
    out = np.zeros((3, len(targets)))
    src_sets = [
        (pos, q, False),
        (np.stack([pos[0], pos[1], -pos[2]]), s[0] * q, True),
        (np.stack([pos[0], pos[1], 2.0 * L[2] - pos[2]]), s[1] * q, True),
    ]
    chunk = max(1, 4_000_000 // max(n, 1))
    for c0 in range(0, len(targets), chunk):
        ti = targets[c0:c0 + chunk]
        xi = pos[:, ti]
        for spos, sq, is_image in src_sets:
            d = xi[:, :, None] - spos[:, None, :]
            d[0] -= L[0] * np.round(d[0] / L[0])
            d[1] -= L[1] * np.round(d[1] / L[1])
            r = np.sqrt((d * d).sum(axis=0))
            # a pair at zero separation (an ion exactly on a wall and its own
            # image, or two coincident ions) has no direction and is skipped
            mask = (r < psi) & (r > 0.0)
            if not is_image:
                mask[np.arange(len(ti)), ti] = False
            rr = np.where(mask, r, 1.0)
            g = table_lookup(table, dr, rr / h)
            mag = np.where(mask, (q[ti][:, None] * sq[None, :]) / (4.0 * np.pi * eps)
                           * (1.0 / rr ** 2 - g / h ** 2) / rr, 0.0)
            out[:, c0:c0 + len(ti)] += (mag[None] * d).sum(axis=2)
    return out


def _pair_force(grid, eps, psi, table, dr, q_a, q_b, d):
    """P3M pair correction on separations d [3, m] (minimum image applied here);
    returns (mask of pairs with 0 < r < psi, force on a for those pairs)."""
    L, h = grid.L, grid.h
    d = d.copy()
    d[0] -= L[0] * np.round(d[0] / L[0])
    d[1] -= L[1] * np.round(d[1] / L[1])
    r = np.sqrt((d * d).sum(axis=0))
    ok = (r < psi) & (r > 0.0)
    r, d = r[ok], d[:, ok]
    g = table_lookup(table, dr, r / h)
    mag = (q_a[ok] * q_b[ok]) / (4.0 * np.pi * eps) * (1.0 / r ** 2 - g / h ** 2) / r
    return ok, mag * d


def _near_field_targets(grid, pos, q, eps, psi, table, dr, bc_types, targets):
    """near_field_pairs for the ions `targets` only (tree of all ions, ball queries)."""
    from scipy.spatial import cKDTree
    L = grid.L
    t = np.asarray(targets)
    out = np.zeros((3, len(t)))
    pts = pos.T.copy()
    pts[:, 0] = np.mod(pts[:, 0], L[0])
    pts[:, 1] = np.mod(pts[:, 1], L[1])
    box = [L[0], L[1], 4.0 * L[2] + 8.0 * psi]
    off = 2.0 * psi  # keep every point set inside the tree box in z
    s = (source_image_signs(grid, pos, bc_types[0]), source_image_signs(grid, pos, bc_types[1]))
    sets = [(pts, np.arange(pos.shape[1]), np.ones(pos.shape[1]))]
    for wall in (0, 1):
        idx = np.nonzero(pos[2] < psi if wall == 0 else pos[2] > L[2] - psi)[0]
        img = pts[idx].copy()
        img[:, 2] = -img[:, 2] if wall == 0 else 2.0 * L[2] - img[:, 2]
        sets.append((img, idx, s[wall][idx]))
    for src, ids, sign in sets:
        if len(ids) == 0:
            continue
        shifted = src.copy()
        shifted[:, 2] += off
        tq = pts[t].copy()
        tq[:, 2] += off
        lists = cKDTree(shifted, boxsize=box).query_ball_point(tq, psi)
        a = np.repeat(np.arange(len(t)), [len(x) for x in lists])
        if len(a) == 0:
            continue
        b = np.concatenate([np.asarray(x, dtype=np.int64) for x in lists])
        d = pos[:, t[a]] - np.stack([pos[0, ids[b]], pos[1, ids[b]], src[b, 2]])
        ok, f = _pair_force(grid, eps, psi, table, dr, q[t[a]], sign[b] * q[ids[b]], d)
        for k in range(3):
            np.add.at(out[k], a[ok], f[k])
    return out


def near_field_pairs(grid, pos, q, eps, psi, table, dr, bc_types, targets=None):
    """The same correction as near_field, with the candidate pairs found by a k-d tree
    (scipy cKDTree, periodic in x and y) instead of brute force; the wall images are
    taken among the ions closer than psi to a wall.  With `targets` the forces of
    that subset only (each found by a ball query against all ions and images)."""
    from scipy.spatial import cKDTree
    if targets is not None:
        return _near_field_targets(grid, pos, q, eps, psi, table, dr, bc_types, targets)
    L = grid.L
    h = grid.h
    n = pos.shape[1]
    out = np.zeros((3, n))
    pts = pos.T.copy()
    pts[:, 0] = np.mod(pts[:, 0], L[0])
    pts[:, 1] = np.mod(pts[:, 1], L[1])
    tree = cKDTree(pts, boxsize=[L[0], L[1], 4.0 * L[2] + 4.0 * psi])
    pairs = tree.query_pairs(psi, output_type="ndarray")
    if len(pairs):
        i, j = pairs[:, 0], pairs[:, 1]
        d = pos[:, i] - pos[:, j]
        d[0] -= L[0] * np.round(d[0] / L[0])
        d[1] -= L[1] * np.round(d[1] / L[1])
        r = np.sqrt((d * d).sum(axis=0))
        ok = (r < psi) & (r > 0.0)
        i, j, d, r = i[ok], j[ok], d[:, ok], r[ok]
        g = table_lookup(table, dr, r / h)
        mag = (q[i] * q[j]) / (4.0 * np.pi * eps) * (1.0 / r ** 2 - g / h ** 2) / r
        for k in range(3):
            np.add.at(out[k], i, mag * d[k])
            np.add.at(out[k], j, -mag * d[k])
    s = (source_image_signs(grid, pos, bc_types[0]), source_image_signs(grid, pos, bc_types[1]))
    for wall, near in ((0, pos[2] < psi), (1, pos[2] > L[2] - psi)):
        idx = np.nonzero(near)[0]
        if len(idx) == 0:
            continue
        sub = pts[idx].copy()
        img = sub.copy()
        img[:, 2] = -sub[:, 2] if wall == 0 else 2.0 * L[2] - sub[:, 2]
        off = 2.0 * psi  # keep both point sets inside the tree box in z
        sub[:, 2] += off
        img[:, 2] += off
        box = [L[0], L[1], 4.0 * L[2] + 8.0 * psi]
        sm = cKDTree(sub, boxsize=box).sparse_distance_matrix(
            cKDTree(img, boxsize=box), psi, output_type="ndarray")
        if len(sm) == 0:
            continue
        a, b = idx[sm["i"]], idx[sm["j"]]
        zimg = -pos[2, b] if wall == 0 else 2.0 * L[2] - pos[2, b]
        d = np.stack([pos[0, a] - pos[0, b], pos[1, a] - pos[1, b], pos[2, a] - zimg])
        d[0] -= L[0] * np.round(d[0] / L[0])
        d[1] -= L[1] * np.round(d[1] / L[1])
        r = np.sqrt((d * d).sum(axis=0))
        ok = (r < psi) & (r > 0.0)
        a, b, d, r = a[ok], b[ok], d[:, ok], r[ok]
        g = table_lookup(table, dr, r / h)
        mag = (q[a] * (s[wall][b] * q[b])) / (4.0 * np.pi * eps) * (1.0 / r ** 2 - g / h ** 2) / r
        for k in range(3):
            np.add.at(out[k], a, mag * d[k])
    return out


def periodic_poisson(grid, eps, rho):
    """-eps lap_h phi = rho on a triply periodic grid (mean-zero gauge); used only
    to tabulate the free-space grid pair force."""
    nx, ny, nz, h = grid.nx, grid.ny, grid.nz, grid.h
    R = np.fft.fftn(rho)
    k2 = (4.0 / h ** 2) * (np.sin(np.pi * np.arange(nz) / nz)[:, None, None] ** 2
                           + np.sin(np.pi * np.arange(ny) / ny)[None, :, None] ** 2
                           + np.sin(np.pi * np.arange(nx) / nx)[None, None, :] ** 2)
    k2[0, 0, 0] = 1.0
    P = R / (eps * k2)
    P[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(P))


def periodic_grid_field(grid, pos, phi):
    """J^es(-grad_h phi) for a triply periodic cell-centred phi."""
    nz = grid.nz
    depth = 3
    ext = np.concatenate([phi[nz - depth:], phi, phi[:depth]], axis=0)
    ex, ey, ez = face_fields(grid, ext, depth)
    p = pos.copy()
    return np.stack([
        _gather(grid, p, ex, (0.0, 0.5, 0.5), depth),
        _gather(grid, p, ey, (0.5, 0.0, 0.5), depth),
        _gather(grid, p, ez, (0.5, 0.5, 0.0), depth),
    ])


def spread_periodic(grid, pos, w):
    """S on a triply periodic grid (no walls); used only for the pair-force table."""
    nx, ny, nz, h = grid.nx, grid.ny, grid.nz, grid.h
    ix, wx = node_weights(pos[0], h, 0.5, nx)
    iy, wy = node_weights(pos[1], h, 0.5, ny)
    iz, wz = node_weights(pos[2], h, 0.5, nz)
    out = np.zeros((nz, ny, nx))
    w = np.asarray(w, dtype=np.float64)
    for c in range(5):
        for b in range(5):
            for a in range(5):
                np.add.at(out, (iz[:, c], iy[:, b], ix[:, a]),
                          w * wx[:, a] * wy[:, b] * wz[:, c] / h ** 3)
    return out

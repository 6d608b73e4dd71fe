"""Energy and electro-osmotic-flux functionals of the electrostatic pass and their
gradients (the adjoint, a project addition on Sec. II.B.1 and Sec. II.D stages 1-2).

Part of the test oracle (test infrastructure only): plain FP64 numpy; the reverse
sweep is written out operator by operator, in the order of the forward pass.

Forward (the readings used by both implementations):
  rho = S q + b        S the folded charge spreading (eq kernel2, Fig. folded), b the
                       wall terms of the inhomogeneous conditions (bc_rhs)
  phi = A^+ rho        A = -eps lap_h with homogeneous ghosts (symmetric; the
                       pseudo-inverse, mean(phi) = 0, when both walls are Neumann)
  E_i = J^es(-grad_h phi_ext)(x_i),  phi_ext = phi with the wall ghosts (eq efieldop)
  F_x,i = q_i (E_x,i + E_ext,x)
  U = (1/2) dV <rho, phi>            electrostatic energy of charges and wall sources
  Q = sum_i w(z_i) F_x,i             mean electro-osmotic flux velocity

U differs from dV [rho_q^T A^-1 rho_q / 2 + rho_q^T A^-1 b] (rho_q = S q) by the
constant dV b^T A^+ b / 2, so its gradients in x and q are the same; its gradient in
the wall field is dV B^T phi (B: field -> b).  Q is the channel mean of the x
velocity of the no-slip Stokes flow driven by S^hy F_x: only the kappa = 0 mode of
the x momentum equation survives the mean, so with
  -eta D_zz g = 1 / nz   (no-slip ghosts g_{-1} = -g_0, g_nz = -g_{nz-1})
the weight is w(z) = (1 / (nx ny h^3)) sum_k s_k g_k wz_k(z), wz the cell-height
kernel weights in z and s the no-slip image sign (-1 below / above the walls).
"""
import numpy as np

from . import electrostatics as es
from .peskin import node_weights_grad


def poiseuille_profile(grid, eta):
    """g of -eta D_zz g = 1/nz with the no-slip ghosts (dense solve)."""
    nz, h = grid.nz, grid.h
    A = (2.0 * np.eye(nz) - np.eye(nz, k=1) - np.eye(nz, k=-1)) * (eta / h ** 2)
    A[0, 0] += eta / h ** 2    # ghost g_{-1} = -g_0
    A[-1, -1] += eta / h ** 2  # ghost g_nz = -g_{nz-1}
    return np.linalg.solve(A, np.full(nz, 1.0 / nz))


def eo_weight(grid, z, eta):
    """w(z) and dw/dz for the ions' heights z."""
    nz = grid.nz
    g = poiseuille_profile(grid, eta)
    iz, wz, dwz = node_weights_grad(z, grid.h, 0.5)
    s = np.ones_like(wz)
    lo, hi = iz < 0, iz >= nz
    s[lo | hi] = -1.0
    k = np.where(lo, -1 - iz, np.where(hi, 2 * nz - 1 - iz, iz))
    norm = 1.0 / (grid.nx * grid.ny * grid.h ** 3)
    w = norm * (s * g[k] * wz).sum(axis=1)
    dw = norm * (s * g[k] * dwz).sum(axis=1)
    return w, dw


def forward(grid, pos, q, p):
    """(U, Q, state) for the electrostatic pass of positions `pos` and charges `q`."""
    eps, bct, bcv = p["eps"], p["bc_types"], p["bc_values"]
    rho = es.spread_charge(grid, pos, q, bct) + es.bc_rhs(grid, eps, bct, bcv)
    phi = es.solve_poisson(grid, eps, bct, rho)
    ext = es.ghost_extend(grid, eps, bct, bcv, phi)
    ex, ey, ez = es.face_fields(grid, ext)
    E = es.interp_field(grid, pos, ex, ey, ez)
    Fx = q * (E[0] + p["e_ext"][0])
    w, dw = eo_weight(grid, pos[2], p["eta"])
    U = 0.5 * grid.dV * float((rho * phi).sum())
    Q = float((w * Fx).sum())
    return U, Q, dict(rho=rho, phi=phi, ex=ex, E=E, Fx=Fx, w=w, dw=dw)


def energy(grid, pos, q, p):
    return forward(grid, pos, q, p)[0]


def flux(grid, pos, q, p):
    return forward(grid, pos, q, p)[1]


def _gather_value_grad(grid, pos, field_ext, offsets, depth=3):
    """sum_n W_n(x_i) f_n and its gradient in x_i over the ghost-extended field."""
    nx, ny, h = grid.nx, grid.ny, grid.h
    ix, wx, dx = node_weights_grad(pos[0], h, offsets[0], nx)
    iy, wy, dy = node_weights_grad(pos[1], h, offsets[1], ny)
    iz, wz, dz = node_weights_grad(pos[2], h, offsets[2])
    iz = iz + depth
    val = np.zeros(pos.shape[1])
    grad = np.zeros((3, pos.shape[1]))
    for c in range(5):
        for b in range(5):
            for a in range(5):
                f = field_ext[iz[:, c], iy[:, b], ix[:, a]]
                val += wx[:, a] * wy[:, b] * wz[:, c] * f
                grad[0] += dx[:, a] * wy[:, b] * wz[:, c] * f
                grad[1] += wx[:, a] * dy[:, b] * wz[:, c] * f
                grad[2] += wx[:, a] * wy[:, b] * dz[:, c] * f
    return val, grad


def _homogeneous(grid, p, f):
    """f with the wall ghosts of the homogeneous conditions (the folds of S)."""
    return es.ghost_extend(grid, p["eps"], p["bc_types"], (None, None), f)


def _scatter_ex(grid, pos, lam, depth=3):
    """Transpose of the E_x gather: per-ion lam onto the ghost-extended x-face grid."""
    nx, ny, nz, h = grid.nx, grid.ny, grid.nz, grid.h
    out = np.zeros((nz + 2 * depth, ny, nx))
    ix, wx, _ = node_weights_grad(pos[0], h, 0.0, nx)
    iy, wy, _ = node_weights_grad(pos[1], h, 0.5, ny)
    iz, wz, _ = node_weights_grad(pos[2], h, 0.5)
    iz = iz + depth
    for c in range(5):
        for b in range(5):
            for a in range(5):
                np.add.at(out, (iz[:, c], iy[:, b], ix[:, a]), lam * wx[:, a] * wy[:, b] * wz[:, c])
    return out


def gradients(grid, pos, q, p, gU=1.0, gQ=1.0, depth=3, targets=None):
    """gU dU + gQ dQ with respect to positions [3, n], charges [n], the two wall
    fields ([ny, nx] each) and the applied field [3].  With `targets` the position
    and charge gradients are those of that subset of ions only."""
    eps, bct = p["eps"], p["bc_types"]
    nz, h = grid.nz, grid.h
    U, Q, st = forward(grid, pos, q, p)
    phi, ex, Fx, w, dw = st["phi"], st["ex"], st["Fx"], st["w"], st["dw"]
    Ex = st["E"][0]
    # --- Q -> E_x at the ions -> face values -> ghost-extended phi ---
    lam = gQ * w * q
    lam_face = _scatter_ex(grid, pos, lam, depth)
    # ex(face i) = -(phi_ext(i) - phi_ext(i-1)) / h
    lam_ext = (-lam_face + np.roll(lam_face, -1, axis=2)) / h
    # ghost-extended phi -> phi and the wall fields
    lam_phi = lam_ext[depth:depth + nz].copy()
    dbc = [np.zeros((grid.ny, grid.nx)), np.zeros((grid.ny, grid.nx))]
    for m in range(depth):
        for wall in (0, 1):
            dst = depth - 1 - m if wall == 0 else depth + nz + m
            src = m if wall == 0 else nz - 1 - m
            if bct[wall] == es.DIRICHLET:
                lam_phi[src] -= lam_ext[dst]      # 2 phi_b - phi_m
                dbc[wall] += 2.0 * lam_ext[dst]
            else:
                lam_phi[src] += lam_ext[dst]      # phi_m + (2m+1) h sigma / eps
                dbc[wall] += (2 * m + 1) * h / eps * lam_ext[dst]
    # --- phi = A^+ rho (A symmetric): the adjoint solve ---
    mu = es.solve_poisson(grid, eps, bct, lam_phi, project=True)
    # --- rho = S q + b: cotangent gU dV phi + mu on rho ---
    rbar = gU * grid.dV * phi + mu
    for wall, layer in ((0, 0), (1, nz - 1)):
        coef = 2.0 * eps / h ** 2 if bct[wall] == es.DIRICHLET else 1.0 / h
        dbc[wall] += coef * rbar[layer]
    de = np.array([gQ * float((q * w).sum()), 0.0, 0.0])
    sel = slice(None) if targets is None else np.asarray(targets)
    pos, q, w, dw, Fx, Ex = pos[:, sel], q[sel], w[sel], dw[sel], Fx[sel], Ex[sel]
    # S^T rbar at the ions (value and gradient): J with the homogeneous ghosts / dV
    val, grad = _gather_value_grad(grid, pos, _homogeneous(grid, p, rbar), (0.5, 0.5, 0.5), depth)
    dq = val / grid.dV
    dpos = q[None, :] * grad / grid.dV
    # --- F_x = q (E_x + E_ext,x) and w(z) ---
    dq += gQ * w * (Ex + p["e_ext"][0])
    _, gEx = _gather_value_grad(grid, pos, ex, (0.0, 0.5, 0.5), depth)
    dpos += (gQ * w * q)[None, :] * gEx
    dpos[2] += gQ * dw * Fx
    return dict(U=U, Q=Q, pos=dpos, q=dq, bc=dbc, e_ext=de)

"""Pins of the oracle's energy / electro-osmotic-flux gradients (CPU only).

  * the kernel derivative: finite differences and the discrete moment identities
    sum_j phi'(z - j) = 0 and sum_j (z - j) phi'(z - j) = -1 (derivatives of the
    partition of unity and first-moment conditions of App. B);
  * the flux weight w(z): equal to the channel-mean velocity of the full no-slip
    Stokes solve for a unit x force (a different code path), and to the continuous
    plane-Poiseuille result z (Lz - z) / (2 eta Lz Lx Ly) up to O(h^2);
  * U is quadratic and Q affine or quadratic in the charges, the wall fields and
    E_ext, so central differences along random directions are exact up to
    rounding: every non-position gradient is pinned to ~1e-9;
  * position gradients against central differences with step 1e-6 on 4,096 ions
    (the kernel is C^1 with kinks in its second derivative, so O(step) agreement);
  * shift invariance: a uniform change of one wall field leaves every x force and
    hence Q unchanged, so the wall gradient of Q sums to zero on each wall;
  * -dU/dx equals the forward electrostatic force up to the discretisation gap
    between J(grad_h phi) and grad(J phi).
"""
import numpy as np
import pytest

from oracle import adjoint, electrostatics as es, stokes
from oracle.peskin import dphi_pe, phi_pe
import workloads

D, N = es.DIRICHLET, es.NEUMANN


def _case(bc, nx=16, ny=16, nz=16, n=200, seed=3):
    grid = es.Grid(nx, ny, nz)
    rng = np.random.default_rng(seed)
    pos, q = workloads.random_ions(nx, ny, nz, n, seed)
    pos[2, :n // 8] = rng.uniform(0.0, 2.5, n // 8)            # within the ghost reach
    pos[2, n // 8:n // 4] = nz - rng.uniform(0.0, 2.5, n // 4 - n // 8)
    bcv = [rng.normal(scale=0.3, size=(ny, nx)) for _ in range(2)]
    if bc == (N, N):
        # neutral: sum q + h^2 (sum sigma_lo + sum sigma_hi) = 0
        shift = (q.sum() + grid.h ** 2 * (bcv[0].sum() + bcv[1].sum())) / (2 * nx * ny * grid.h ** 2)
        bcv = [b - shift for b in bcv]
    p = dict(eps=1.0 / (4 * np.pi * 4.46), bc_types=bc, bc_values=tuple(bcv),
             e_ext=np.array([0.1, 0.0, 0.0]), eta=1.0 / (6 * np.pi))
    return grid, pos, q, p


def _neutral_dirs(rng, shape, count):
    v = rng.normal(size=(count,) + shape)
    return v


def test_kernel_derivative():
    z = np.linspace(-2.6, 2.6, 20001)
    off = np.abs(np.abs(z) - np.round(np.abs(z))) > 1e-3
    e = 1e-6
    fd = (phi_pe(z[off] + e) - phi_pe(z[off] - e)) / (2 * e)
    assert np.abs(fd - dphi_pe(z[off])).max() < 1e-8
    x = np.random.default_rng(0).uniform(0, 1, 500)
    j = np.arange(-3, 4)
    d = dphi_pe(x[:, None] - j[None, :])
    np.testing.assert_allclose(d.sum(1), 0.0, atol=1e-14)
    np.testing.assert_allclose(((x[:, None] - j) * d).sum(1), -1.0, atol=1e-14)


def test_flux_weight_is_the_mean_stokes_velocity():
    grid = es.Grid(8, 8, 12, h=0.9)
    eta = 0.37
    pts = np.array([[1.3, 4.4, 0.2], [6.1, 2.9, 5.4], [3.3, 7.7, 10.6], [2.2, 0.4, 9.1]]).T
    w, _ = adjoint.eo_weight(grid, pts[2], eta)
    for i in range(pts.shape[1]):
        F = np.zeros((3, 1))
        F[0, 0] = 1.0
        fx, fy, fz = stokes.spread_force(grid, pts[:, i:i + 1], F)
        u, v, wv, _ = stokes.solve_stokes(grid, eta, fx, fy, fz)
        assert abs(u.mean() - w[i]) < 1e-12 * abs(w[i])


def test_flux_weight_matches_continuous_poiseuille():
    grid = es.Grid(16, 16, 64)
    eta = 0.5
    z = np.linspace(8.0, 56.0, 25)
    w, dw = adjoint.eo_weight(grid, z, eta)
    L = grid.L
    cont = z * (L[2] - z) / (2 * eta * L[2] * L[0] * L[1])
    np.testing.assert_allclose(w, cont, rtol=2e-3)
    dcont = (L[2] - 2 * z) / (2 * eta * L[2] * L[0] * L[1])
    np.testing.assert_allclose(dw, dcont, atol=2e-3 * np.abs(cont).max() / L[2])


@pytest.mark.parametrize("bc", [(D, D), (N, N), (D, N)])
def test_polynomial_directions_are_exact(bc):
    grid, pos, q, p = _case(bc)
    g = adjoint.gradients(grid, pos, q, p, gU=0.7, gQ=1.3)
    fun = lambda pp, qq, P: 0.7 * adjoint.energy(grid, pp, qq, P) + 1.3 * adjoint.flux(grid, pp, qq, P)
    rng = np.random.default_rng(9)
    t = 1e-2
    # charges (neutral direction, so the all-Neumann problem stays solvable)
    v = rng.normal(size=q.shape)
    v -= v.mean()
    fd = (fun(pos, q + t * v, p) - fun(pos, q - t * v, p)) / (2 * t)
    an = float(g["q"] @ v)
    assert abs(fd - an) < 1e-9 * (abs(an) + np.abs(g["q"]).sum() * np.abs(v).max() * 1e-3)
    # wall fields (a direction of zero total, for the same reason)
    vb = [rng.normal(size=b.shape) for b in p["bc_values"]]
    tot = (vb[0].sum() + vb[1].sum()) / (2 * vb[0].size)
    vb = [b - tot for b in vb]
    def with_bc(s):
        P = dict(p)
        P["bc_values"] = tuple(b + s * d for b, d in zip(p["bc_values"], vb))
        return P
    fd = (fun(pos, q, with_bc(t)) - fun(pos, q, with_bc(-t))) / (2 * t)
    an = float((g["bc"][0] * vb[0]).sum() + (g["bc"][1] * vb[1]).sum())
    assert abs(fd - an) < 1e-9 * max(abs(an), 1e-3 * sum(np.abs(x).sum() for x in g["bc"]))
    # applied field
    for k in range(3):
        def with_e(s):
            P = dict(p)
            e = np.array(p["e_ext"], dtype=float)
            e[k] += s
            P["e_ext"] = e
            return P
        fd = (fun(pos, q, with_e(t)) - fun(pos, q, with_e(-t))) / (2 * t)
        assert abs(fd - g["e_ext"][k]) < 1e-9 * max(abs(g["e_ext"][0]), 1e-12)


@pytest.mark.parametrize("bc", [(D, D), (N, N)])
def test_wall_gradient_of_flux_sums_to_zero(bc):
    grid, pos, q, p = _case(bc)
    g = adjoint.gradients(grid, pos, q, p, gU=0.0, gQ=1.0)
    for wall in (0, 1):
        a = g["bc"][wall]
        assert abs(a.sum()) < 1e-12 * np.abs(a).sum()
        assert np.abs(a).max() > 0


@pytest.mark.parametrize("bc", [(D, D), (N, N), (D, N)])
def test_position_gradient_small_case(bc):
    grid, pos, q, p = _case(bc, n=120, seed=4)
    g = adjoint.gradients(grid, pos, q, p, gU=1.0, gQ=2.0)
    fun = lambda pp: adjoint.energy(grid, pp, q, p) + 2.0 * adjoint.flux(grid, pp, q, p)
    e = 1e-6
    for i in (0, 1, 20, 60, 119):  # near-wall and bulk ions
        for k in range(3):
            d = np.zeros_like(pos)
            d[k, i] = e
            fd = (fun(pos + d) - fun(pos - d)) / (2 * e)
            assert abs(fd - g["pos"][k, i]) < 1e-5 * (abs(g["pos"][k, i]) + 1e-2), (i, k)


def test_position_gradient_4096_ions():
    """Central differences with step 1e-6 on the 4,096-ion, 32^3 dielectric case."""
    w = workloads.WORKLOADS["dielectric_32x32x32_n4096"]
    P = workloads.make_params(w)
    pos, q, ids, species = workloads.make_ions(w)
    grid = es.Grid(w.nx, w.ny, w.nz, w.h)
    p = dict(eps=P["eps"], bc_types=P["bc_types"], bc_values=P["bc_values"], e_ext=P["e_ext"],
             eta=P["eta"])
    g = adjoint.gradients(grid, pos, q, p, gU=1.0, gQ=1.0)
    fun = lambda pp: adjoint.energy(grid, pp, q, p) + adjoint.flux(grid, pp, q, p)
    rng = np.random.default_rng(2)
    e = 1e-6
    for _ in range(3):
        v = rng.normal(size=pos.shape)
        v /= np.linalg.norm(v)
        fd = (fun(pos + e * v) - fun(pos - e * v)) / (2 * e)
        an = float((g["pos"] * v).sum())
        assert abs(fd - an) < 1e-5 * np.linalg.norm(g["pos"]), (fd, an)


def _pair_gap(nn, spacing):
    """Relative gap between -dU/dx and the forward force F^P, each without the ion's
    single-ion part (its self and own-image terms, which differ between
    grad(J phi) and J(grad_h phi) by lattice artefacts of order one)."""
    grid = es.Grid(nn, nn, nn)
    eps = 1.0 / (4 * np.pi * 4.46)
    rng = np.random.default_rng(1)
    ax = np.arange(spacing / 2, nn, spacing)
    X, Y, Z = np.meshgrid(ax, ax, ax[(ax >= 2) & (ax <= nn - 2)], indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), Z.ravel()]) + rng.uniform(-0.4, 0.4, (3, X.size))
    q = np.where(rng.uniform(size=X.size) < 0.5, 1.0, -1.0)
    p = dict(eps=eps, bc_types=(D, D), bc_values=(None, None), e_ext=np.zeros(3), eta=1.0)
    gU = adjoint.gradients(grid, pos, q, p, 1.0, 0.0)["pos"]
    F = es.grid_force(grid, pos, q, eps, (D, D), (None, None))[3]
    for i in range(pos.shape[1]):
        one = pos[:, i:i + 1]
        gU[:, i] -= adjoint.gradients(grid, one, q[i:i + 1], p, 1.0, 0.0)["pos"][:, 0]
        F[:, i] -= es.grid_force(grid, one, q[i:i + 1], eps, (D, D), (None, None))[3][:, 0]
    return np.linalg.norm(-gU - F) / np.linalg.norm(F)


def test_energy_gradient_is_minus_the_force():
    """Measured pair gap: ~3.0e-2 at a 4 h ion spacing, ~1.3e-2 at 8 h."""
    g4 = _pair_gap(16, 4)
    g8 = _pair_gap(32, 8)
    assert g4 < 4e-2 and g8 < 2e-2 and g8 < g4, (g4, g8)

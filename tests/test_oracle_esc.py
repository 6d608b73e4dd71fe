"""Pins of the oracle's ESC kernel (App. B, eq eskernel) and of its per-ion hydrodynamic
spread / interpolation (CPU only).
  * the normalisation by adaptive quadrature equals an independent Gauss-Legendre rule
    in theta (zeta = alpha sin theta); beta = 0 is the box kernel, exactly; for large
    beta the integral follows the Laplace expansion alpha sqrt(2 pi / beta)(1 - 3/(8 beta));
  * the kernel is even, positive on its support and zero outside;
  * the per-ion spread with every kernel w = 0 is the 4-point Peskin spread;
  * S^hy and J^hy with ESC kernels are adjoint (walls included), and an ion on a wall
    spreads nothing (no-slip folds)."""
import numpy as np
import pytest

from oracle import electrostatics as es, esc, stokes

KERNELS = [(7, 7.0), (4, 8.0), (5, 3.0), (8, 12.0), (6, 0.0)]


@pytest.mark.parametrize("kern", KERNELS)
def test_normalisation_two_quadratures(kern):
    w, beta = kern
    a = 0.5 * w
    t, wt = np.polynomial.legendre.leggauss(120)
    th = 0.5 * np.pi * t
    gl = a * 0.5 * np.pi * np.sum(wt * np.exp(beta * (np.cos(th) - 1.0)) * np.cos(th))
    assert abs(esc.esc_norm(w, beta) - gl) <= 1e-13 * gl


def test_box_and_laplace_limits():
    for w in (4, 5, 7, 8):
        assert abs(esc.esc_norm(w, 0.0) - w) < 1e-13
        z = np.linspace(-0.499 * w, 0.499 * w, 41)
        np.testing.assert_allclose(esc.phi_esc(z, w, 0.0), 1.0 / w, rtol=1e-13)
    w, beta = 8, 400.0
    a = 0.5 * w
    approx = a * np.sqrt(2.0 * np.pi / beta) * (1.0 - 3.0 / (8.0 * beta))
    assert abs(esc.esc_norm(w, beta) / approx - 1.0) < 1e-4


@pytest.mark.parametrize("kern", KERNELS)
def test_shape(kern):
    w, beta = kern
    z = np.linspace(-0.5 * w + 1e-9, 0.5 * w - 1e-9, 301)
    v = esc.phi_esc(z, w, beta)
    np.testing.assert_array_equal(v, esc.phi_esc(-z, w, beta))
    assert np.all(v > 0.0)
    outside = np.array([-0.5 * w - 1e-9, 0.5 * w, 0.5 * w + 0.3, -w])
    assert np.all(esc.phi_esc(outside, w, beta) == 0.0)


def _ions(grid, n, seed):
    rng = np.random.default_rng(seed)
    pos = np.empty((3, n))
    pos[0] = rng.uniform(0, grid.L[0], n)
    pos[1] = rng.uniform(0, grid.L[1], n)
    pos[2] = rng.uniform(0, grid.L[2], n)
    pos[2, :n // 4] = rng.uniform(0.0, 1.5, n // 4)
    pos[2, 0], pos[2, 1] = 0.0, grid.L[2]
    return pos


def test_peskin_kernels_reproduce_the_peskin_spread():
    grid = es.Grid(8, 8, 9)
    pos = _ions(grid, 40, 1)
    F = np.random.default_rng(2).normal(size=(3, 40))
    ref = stokes.spread_force(grid, pos, F)
    got = stokes.spread_force_kernels(grid, pos, F, np.zeros((40, 2)))
    for a, b in zip(got, ref):
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


def test_esc_spread_interp_adjoint_and_wall():
    grid = es.Grid(8, 8, 10)
    n = 30
    pos = _ions(grid, n, 3)
    rng = np.random.default_rng(4)
    F = rng.normal(size=(3, n))
    kern = np.array([KERNELS[i % len(KERNELS)] for i in range(n)], dtype=np.float64)
    f = stokes.spread_force_kernels(grid, pos, F, kern)
    u = rng.normal(size=(10, 8, 8))
    v = rng.normal(size=(10, 8, 8))
    w = rng.normal(size=(11, 8, 8))
    w[0] = 0.0
    w[-1] = 0.0
    J = stokes.interp_velocity_kernels(grid, pos, u, v, w, kern)
    h3 = grid.h ** 3
    lhs = h3 * ((f[0] * u).sum() + (f[1] * v).sum() + (f[2] * w).sum())
    rhs = (F * J).sum()
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + abs(rhs))
    # an ion on a wall spreads nothing
    wall = np.array([[3.3, 5.1], [4.7, 2.2], [0.0, 10.0]])
    g = stokes.spread_force_kernels(grid, wall, np.ones((3, 2)), np.array([[7, 7.0], [4, 8.0]]))
    for a in g:
        assert np.abs(a).max() < 1e-15

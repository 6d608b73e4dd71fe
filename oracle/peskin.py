"""4-point Peskin kernel, written from the paper's App. B (eq peskin1d, eq pkernel).

Part of the test oracle (test infrastructure only).

The 1-D kernel is phi(zeta) with zeta the separation in units of the grid
spacing; the kernel used for spreading / interpolation in one dimension is
phi(zeta) / dr, and the 3-D kernel is the tensor product of three of them.
"""
import numpy as np


def phi_pe(zeta):
    """Dimensionless 1-D 4-point Peskin kernel, eq peskin1d times dr.

    Three branches on r = |zeta|: r <= 1, 1 < r <= 2 and r > 2.
    """
    r = np.abs(np.asarray(zeta, dtype=np.float64))
    out = np.zeros_like(r)
    inner = r <= 1.0
    outer = (r > 1.0) & (r <= 2.0)
    ri = r[inner]
    out[inner] = (3.0 - 2.0 * ri + np.sqrt(1.0 + 4.0 * ri - 4.0 * ri * ri)) / 8.0
    ro = r[outer]
    # the radicand is >= 0 on (1, 2]; clip tiny negative rounding at the ends
    rad = np.maximum(-7.0 + 12.0 * ro - 4.0 * ro * ro, 0.0)
    out[outer] = (5.0 - 2.0 * ro - np.sqrt(rad)) / 8.0
    return out


def node_weights(x, h, offset, period=None):
    """Nodes and 1-D weights of the kernel centred at positions x.

    The node set is {(n + offset) * h : n integer}.  Returns (n [N, 5] int,
    w [N, 5] float): the five nodes n0 - 2 .. n0 + 2 with n0 = floor(x/h - offset)
    and their weights phi((x - (n + offset) h) / h).  One of the five weights is
    always zero (the kernel has support of width 4).  With `period` the node
    index is wrapped into [0, period).
    """
    x = np.asarray(x, dtype=np.float64)
    s = x / h - offset
    n0 = np.floor(s).astype(np.int64)
    n = n0[:, None] + np.arange(-2, 3)[None, :]
    w = phi_pe(s[:, None] - n)
    if period is not None:
        n = np.mod(n, period)
    return n, w


def dphi_pe(zeta):
    """d phi_pe / d zeta, the derivative of each branch of eq peskin1d (odd in zeta).

    Continuous everywhere (the kernel is C^1); zero for |zeta| >= 2 and at 0.
    """
    z = np.asarray(zeta, dtype=np.float64)
    r = np.abs(z)
    out = np.zeros_like(r)
    inner = r <= 1.0
    outer = (r > 1.0) & (r < 2.0)
    ri = r[inner]
    out[inner] = (-2.0 + (2.0 - 4.0 * ri) / np.sqrt(1.0 + 4.0 * ri - 4.0 * ri * ri)) / 8.0
    ro = r[outer]
    rad = np.maximum(-7.0 + 12.0 * ro - 4.0 * ro * ro, 1e-300)
    out[outer] = (-2.0 - (6.0 - 4.0 * ro) / np.sqrt(rad)) / 8.0
    return np.sign(z) * out


def node_weights_grad(x, h, offset, period=None):
    """As node_weights, plus d w / d x (= dphi_pe(zeta) / h) for each node."""
    x = np.asarray(x, dtype=np.float64)
    s = x / h - offset
    n0 = np.floor(s).astype(np.int64)
    n = n0[:, None] + np.arange(-2, 3)[None, :]
    w = phi_pe(s[:, None] - n)
    dw = dphi_pe(s[:, None] - n) / h
    if period is not None:
        n = np.mod(n, period)
    return n, w, dw

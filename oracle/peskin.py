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

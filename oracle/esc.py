"""Exponential-of-semicircle (ESC) kernel of App. B (eq eskernel), for hydrodynamic
spreading and interpolation with a per-species kernel (TEST INFRASTRUCTURE ONLY:
imported by tests/, never by the product path).

In units of the cell size, with alpha = w / 2 (w the number of points of the kernel's
support) and a shape parameter beta,
    psi(zeta) = exp(beta (sqrt(1 - (zeta / alpha)^2) - 1))   for |zeta| < alpha, else 0,
normalised by its integral: phi(zeta) = psi(zeta) / int psi.  A kernel is the pair
(w, beta); w = 0 stands for the 4-point Peskin kernel of eq peskin1d.
"""
import numpy as np
from scipy.integrate import quad

from .peskin import phi_pe


def psi_esc(zeta, w, beta):
    """Unnormalised ESC profile (zero outside |zeta| < w / 2)."""
    z = np.asarray(zeta, dtype=np.float64)
    a = 0.5 * w
    t = np.clip(z / a, -1.0, 1.0)
    inside = np.abs(z) < a
    return np.where(inside, np.exp(beta * (np.sqrt(1.0 - t * t) - 1.0)), 0.0)


def esc_norm(w, beta):
    """int psi over (-w/2, w/2), by adaptive quadrature."""
    a = 0.5 * w
    val, _ = quad(lambda z: float(psi_esc(z, w, beta)), -a, a, epsabs=0.0, epsrel=2e-14,
                  limit=500)
    return val


def phi_esc(zeta, w, beta):
    """ESC kernel normalised to unit integral."""
    return psi_esc(zeta, w, beta) / esc_norm(w, beta)


def kernel_phi(zeta, kernel):
    """phi of kernel (w, beta); w = 0 is the 4-point Peskin kernel."""
    w, beta = kernel
    if w == 0:
        return phi_pe(zeta)
    return phi_esc(zeta, w, beta)


def node_weights_kernel(x, h, offset, kernel, period=None):
    """Nodes n0 - 4 .. n0 + 4 (n0 = floor(x/h - offset)) and their 1-D weights
    phi((x - (n + offset) h) / h) for one kernel (the window covers supports up to 8
    points; weights outside the support are zero).  With `period` the node index is
    wrapped into [0, period)."""
    x = np.asarray(x, dtype=np.float64)
    s = x / h - offset
    n0 = np.floor(s).astype(np.int64)
    n = n0[:, None] + np.arange(-4, 5)[None, :]
    w = kernel_phi(s[:, None] - n, kernel)
    if period is not None:
        n = np.mod(n, period)
    return n, w


def support(kernel):
    """Half-width of the kernel's support in cells."""
    w, _ = kernel
    return 2.0 if w == 0 else 0.5 * w

"""Discrete-ordinates direction sets, as a caller would hand them to the solver.

These are inputs (unit vectors and weights), not part of the solver's
arithmetic: the solver library and the oracle both receive them through their
argument lists.  Every set is returned as ``dirs`` of shape [N, 3] (unit
vectors; circle sets have z = 0) and ``weights`` of shape [N] summing to 1.
"""
import numpy as np


def circle(n):
    """N directions equally spaced on the unit circle, offset by half a step.

    The half-step offset keeps every direction off the coordinate axes, so
    each direction has nonzero x and y components, as the x-y quadrature sets
    of the paper's Sec. 2.1 do (four quadrants, 4M directions).
    """
    if n < 4 or n % 4:
        raise ValueError("circle quadrature needs N a positive multiple of 4")
    theta = 2.0 * np.pi * (np.arange(n) + 0.5) / n
    dirs = np.stack([np.cos(theta), np.sin(theta), np.zeros(n)], axis=1)
    w = np.full(n, 1.0 / n)
    return dirs, w


def axis4():
    """The four axis-aligned directions +x, +y, -x, -y with weight 1/4 each."""
    dirs = np.array([[1.0, 0, 0], [0, 1.0, 0], [-1.0, 0, 0], [0, -1.0, 0]])
    return dirs, np.full(4, 0.25)


def s2_xy():
    """The S_2 level-symmetric set restricted to the upper hemisphere.

    In x-y geometry the paper projects 3D ordinates onto the plane (Sec. 2.1,
    its Fig. "DOM" right panel shows S_N with N = 2): four directions
    (+-1/sqrt3, +-1/sqrt3) in the plane, each of weight 1/4.  The 3D unit
    vectors are returned with z = +1/sqrt3.
    """
    a = 1.0 / np.sqrt(3.0)
    dirs = np.array([[a, a, a], [-a, a, a], [-a, -a, a], [a, -a, a]])
    return dirs, np.full(4, 0.25)


def sphere_product(n_mu=8, n_phi=12):
    """Product set on the unit sphere: Gauss-Legendre in mu times uniform azimuths.

    mu_a are the n_mu Gauss-Legendre nodes on [-1, 1]; the azimuths are
    phi_b = 2 pi (b + 1/2) / n_phi.  Weight = (w_GL / 2) / n_phi, summing to 1.
    Ordering: mu outer, phi inner.
    """
    mu, wmu = np.polynomial.legendre.leggauss(n_mu)
    phi = 2.0 * np.pi * (np.arange(n_phi) + 0.5) / n_phi
    M, P = np.meshgrid(mu, phi, indexing="ij")
    s = np.sqrt(1.0 - M ** 2)
    dirs = np.stack([s * np.cos(P), s * np.sin(P), M], axis=-1).reshape(-1, 3)
    w = (np.repeat(wmu, n_phi) / 2.0) / n_phi
    return dirs, w

"""Seeded synthetic media: per-cell coefficient fields sampled at cell centres.

Grids are cubic cells of side h = 1/n on [0, 1]^d.  Arrays are indexed
[k, j, i] (z, y, x) in 3D and [j, i] (y, x) in 2D, x fastest, matching the
solver's cell order.  Nothing here evaluates the transport equation.
"""
import numpy as np


def cell_centres(shape):
    """Cell-centre coordinates for a grid of the given (…, ny, nx) shape."""
    axes = [(np.arange(s) + 0.5) / s for s in shape]
    return np.meshgrid(*axes, indexing="ij")


def gaussian_random_field(shape, std, corr_len, rng):
    """Zero-mean stationary Gaussian field with squared-exponential covariance.

    Covariance exp(-r^2 / (2 l^2)).  Spectral synthesis on a periodic grid of
    twice the extent in every axis (so the periodic wrap does not correlate
    opposite edges), white noise shaped by the square root of the covariance's
    spectral density, then the corner block of the requested shape is kept and
    rescaled to exactly zero mean and the requested standard deviation.
    """
    shape = tuple(int(s) for s in shape)
    big = tuple(2 * s for s in shape)
    h = 1.0 / shape[-1]
    noise = rng.standard_normal(big)
    k2 = np.zeros(big)
    for ax, s in enumerate(big):
        f = 2.0 * np.pi * np.fft.fftfreq(s, d=h)
        sh = [1] * len(big)
        sh[ax] = s
        k2 = k2 + (f.reshape(sh)) ** 2
    amp = np.exp(-0.25 * k2 * corr_len ** 2)          # sqrt of exp(-k^2 l^2 / 2)
    field = np.real(np.fft.ifftn(np.fft.fftn(noise) * amp))
    field = field[tuple(slice(0, s) for s in shape)]
    field = field - field.mean()
    sd = field.std()
    if sd > 0:
        field = field * (std / sd)
    return field


def lognormal_field(shape, std, corr_len, rng, median=1.0):
    return median * np.exp(gaussian_random_field(shape, std, corr_len, rng))


def centred_inclusion(n, lo_cell, hi_cell, inside, outside):
    """2D field equal to `inside` on cells [lo, hi)^2 and `outside` elsewhere."""
    f = np.full((n, n), float(outside))
    f[lo_cell:hi_cell, lo_cell:hi_cell] = inside
    return f


def checkerboard(n, blocks, black, white):
    """2D blocks x blocks checkerboard; black where floor(b x) + floor(b y) is even."""
    Y, X = cell_centres((n, n))
    parity = (np.floor(blocks * X).astype(int) + np.floor(blocks * Y).astype(int)) % 2
    return np.where(parity == 0, float(black), float(white)), parity == 0


def gaussian_source(shape, width, centre=0.5):
    """exp(-|x - c|^2 / (2 w^2)) sampled at cell centres (any dimension)."""
    cs = cell_centres(shape)
    r2 = sum((c - centre) ** 2 for c in cs)
    return np.exp(-r2 / (2.0 * width ** 2))


def polynomial_medium(n, rng, degree=None):
    """Random separable polynomial media of the paper's experiments (Sec. 4.1).

    Each of sigma_T and sigma_a is (2 + sum_k c_xk (x-1/2)^k)(2 + sum_k c_yk (y-1/2)^k)
    with c ~ U[-1, 1] and k = 0..degree, degree drawn from {1, 2, 3, 4} unless
    given.  sigma_T is then shifted up so that sigma_T - sigma_a >= 0.2.
    """
    Y, X = cell_centres((n, n))

    def poly():
        d = int(rng.integers(1, 5)) if degree is None else int(degree)
        cx = rng.uniform(-1, 1, d + 1)
        cy = rng.uniform(-1, 1, d + 1)
        px = 2.0 + sum(cx[k] * (X - 0.5) ** k for k in range(d + 1))
        py = 2.0 + sum(cy[k] * (Y - 0.5) ** k for k in range(d + 1))
        return px * py

    st = poly()
    sa = poly()
    gap = (st - sa).min()
    if gap < 0.2:
        st = st + (0.2 - gap)
    return st, sa

"""Named synthetic workloads.

A problem is a plain dict of host arrays:

  dim, n = (nx, ny, nz), dirs [N, 3], weights [N], g, kernel ("auto" |
  "flatland" | "sphere"), sigma_t, sigma_a, q [cells] (x fastest),
  eps (scalar or [cells]), inflow ([2*dim, N, face_cells] or None),
  mgnet = dict(c0, levels, nu_pre, nu_post, nu_coarse, coef_ch, seed),
  solver = dict(restart, rtol, max_iters)

Inflow faces are ordered x-, x+, y-, y+, z-, z+; face cells are ordered with
the lower remaining axis fastest (x faces: y fastest then z; y faces: x then
z; z faces: x then y).  Only entries of incoming directions (u.n < 0) are
meaningful.
"""
import numpy as np

from . import media, quadrature


def _flat(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))


def face_cells(n, dim, face):
    nx, ny, nz = n
    axis = face // 2
    if axis == 0:
        return ny * nz
    if axis == 1:
        return nx * nz
    return nx * ny


def left_unit_inflow(n, dim, dirs, value=1.0):
    """Psi = value on the x = 0 face for directions with u_x > 0, zero elsewhere."""
    N = dirs.shape[0]
    fc = max(face_cells(n, dim, f) for f in range(2 * dim))
    inflow = np.zeros((2 * dim, N, fc))
    inflow[0, dirs[:, 0] > 0, :face_cells(n, dim, 0)] = value
    return inflow


def uniform_inflow(n, dim, dirs, value=1.0):
    """Psi = value on every face for every incoming direction."""
    N = dirs.shape[0]
    fc = max(face_cells(n, dim, f) for f in range(2 * dim))
    return np.full((2 * dim, N, fc), float(value))


def _problem(name, dim, n, dirs, w, g, kernel, st, sa, q, eps, inflow, mg, solver):
    return dict(name=name, dim=dim, n=tuple(int(v) for v in n), dirs=np.asarray(dirs, float),
                weights=np.asarray(w, float), g=float(g), kernel=kernel,
                sigma_t=_flat(st), sigma_a=_flat(sa), q=_flat(q),
                eps=(float(eps) if np.isscalar(eps) else _flat(eps)),
                inflow=None if inflow is None else np.ascontiguousarray(inflow, dtype=np.float64),
                mgnet=mg, solver=solver)


def c1(seed=1001):
    """32^2, 16 circle directions, g = 0, eps = 1, sigma_T = 10 inclusion on cells [12, 20)^2."""
    n = 32
    dirs, w = quadrature.circle(16)
    st = media.centred_inclusion(n, 12, 20, 10.0, 1.0)
    sa = np.full((n, n), 0.1)
    q = media.centred_inclusion(n, 12, 20, 1.0, 0.0)
    mg = dict(c0=16, levels=2, nu_pre=2, nu_post=2, nu_coarse=2, coef_ch=3, seed=seed)
    return _problem("C1", 2, (n, n, 1), dirs, w, 0.0, "flatland", st, sa, q, 1.0, None, mg,
                    dict(restart=20, rtol=1e-8, max_iters=5000))


def c2(s=0, n=128, ndir=32, levels=4, c0=None, seed=2001):
    """128^2, 32 directions, flatland HG g = 0.5, eps = 0.01, lognormal GRF sigma_T, left inflow."""
    rng = np.random.default_rng(2000 + s)
    dirs, w = quadrature.circle(ndir)
    st = media.lognormal_field((n, n), 0.5, 0.1, rng)
    sa = np.full((n, n), 0.05)
    q = np.ones((n, n))
    mg = dict(c0=c0 or ndir, levels=levels, nu_pre=2, nu_post=2, nu_coarse=2, coef_ch=3, seed=seed)
    return _problem("C2", 2, (n, n, 1), dirs, w, 0.5, "flatland", st, sa, q, 0.01,
                    left_unit_inflow((n, n, 1), 2, dirs), mg,
                    dict(restart=30, rtol=1e-6, max_iters=20000))


def c4(n=512, ndir=64, levels=5, c0=None, seed=4001):
    """512^2, 64 directions, g = 0.9, eps = 1e-3, 8x8 checkerboard sigma_T in {1, 100}."""
    dirs, w = quadrature.circle(ndir)
    st, black = media.checkerboard(n, 8, 100.0, 1.0)
    sa = np.full((n, n), 0.01)
    q = black.astype(float)
    mg = dict(c0=c0 or ndir, levels=levels, nu_pre=2, nu_post=2, nu_coarse=2, coef_ch=3, seed=seed)
    return _problem("C4", 2, (n, n, 1), dirs, w, 0.9, "flatland", st, sa, q, 1e-3, None, mg,
                    dict(restart=30, rtol=1e-6, max_iters=20000))


def c5(s=0, n=64, n_mu=8, n_phi=12, levels=4, c0=None, seed=5001):
    """64^3, 96 sphere directions, eq. (hg) with g = 0.8, eps = 1e-2, lognormal sigma_T, Gaussian q."""
    rng = np.random.default_rng(5000 + s)
    dirs, w = quadrature.sphere_product(n_mu, n_phi)
    st = media.lognormal_field((n, n, n), 0.7, 0.15, rng)
    sa = np.full((n, n, n), 0.02)
    q = media.gaussian_source((n, n, n), 0.05)
    N = dirs.shape[0]
    mg = dict(c0=c0 or N // 2, levels=levels, nu_pre=2, nu_post=2, nu_coarse=2, coef_ch=3, seed=seed)
    return _problem("C5", 3, (n, n, n), dirs, w, 0.8, "sphere", st, sa, q, 1e-2, None, mg,
                    dict(restart=20, rtol=1e-6, max_iters=20000))


def p0(s=0, regime="diffusion", n=32, seed=6001):
    """The paper's experimental shape (Sec. 4.1): 32^2 grid, 4 directions, polynomial media.

    regime: "diffusion" (eps = 0.01 (c + 0.1), c ~ U[0, 1]), "transport"
    (eps = 1) or "interface" (eps = 0.01 on the central square
    [0.25, 0.75]^2 and 1 outside).
    """
    rng = np.random.default_rng(6000 + s)
    dirs, w = quadrature.s2_xy()
    st, sa = media.polynomial_medium(n, rng)
    q = np.ones((n, n))
    if regime == "diffusion":
        eps = 0.01 * (rng.uniform() + 0.1)
    elif regime == "transport":
        eps = 1.0
    else:
        Y, X = media.cell_centres((n, n))
        inside = (np.abs(X - 0.5) < 0.25) & (np.abs(Y - 0.5) < 0.25)
        eps = np.where(inside, 0.01, 1.0)
    mg = dict(c0=16, levels=3, nu_pre=2, nu_post=2, nu_coarse=2, coef_ch=3, seed=seed)
    return _problem("P0", 2, (n, n, 1), dirs, w, 0.0, "sphere", st, sa, q, eps,
                    left_unit_inflow((n, n, 1), 2, dirs), mg,
                    dict(restart=30, rtol=1e-6, max_iters=5000))


def c3_request(r, ndir_choices=(16, 32), grid_choices=(64, 128, 256)):
    """One request of the serving stream: grid, directions, eps, g drawn from seed 3000 + r."""
    rng = np.random.default_rng(3000 + r)
    n = int(rng.choice(grid_choices))
    ndir = int(rng.choice(ndir_choices))
    eps = float(10.0 ** rng.uniform(-3.0, 0.0))
    g = float(rng.uniform(0.0, 0.8))
    dirs, w = quadrature.circle(ndir)
    st = media.lognormal_field((n, n), 0.5, 0.1, rng)
    sa = np.full((n, n), 0.05)
    q = np.ones((n, n))
    mg = dict(c0=ndir, levels=4, nu_pre=2, nu_post=2, nu_coarse=2, coef_ch=3,
              seed=3100 + ndir)
    return _problem("C3", 2, (n, n, 1), dirs, w, g, "flatland", st, sa, q, eps,
                    left_unit_inflow((n, n, 1), 2, dirs), mg,
                    dict(restart=30, rtol=1e-6, max_iters=20000))


def c3_arrivals(count=512, rate=1.0, seed=3999):
    """Poisson arrival times (seconds) at `rate` requests per second."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, count))


def problem_weights(problem):
    """(header, tensors) of the seeded MgNet for a problem."""
    from .weights import seeded_weights
    mg = problem["mgnet"]
    return seeded_weights(problem["dim"], problem["dirs"].shape[0], mg["c0"], mg["levels"],
                          mg["nu_pre"], mg["nu_post"], mg["nu_coarse"], mg["coef_ch"], mg["seed"])

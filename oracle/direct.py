"""Independent solvers that pin the oracle's operator and FGMRES (test infrastructure).

None of these is on the solver path; each reaches the same discrete solution
(or a provable limit of it) by a different route:

  dense_matrix / lu_solve    assemble L column by column and factorise
  sweep_solve                transport sweep: exact when there is no scattering
  source_iteration           psi <- T^{-1}(sS S psi + b) with sweeps
  isotropic_limit            the eps -> 0 limit at fixed h of the scalar flux
"""
import numpy as np

from . import discretisation as dsc


def dense_matrix(D):
    """Dense L (n x n, n = N * cells) assembled as columns L e_j.  For n <= 4096."""
    n = D.n
    if n > 4096:
        raise ValueError("dense assembly is for tiny problems only")
    A = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        A[:, j] = dsc.apply_L(D, e).reshape(-1)
        e[j] = 0.0
    return A


def lu_solve(D, b=None):
    b = dsc.rhs(D) if b is None else b
    return np.linalg.solve(dense_matrix(D), np.asarray(b).reshape(-1)).reshape(D.N, D.cells)


def _upwind_order(D, m):
    """Cell visiting order for direction m: every upwind neighbour comes first."""
    rng = []
    for a, n in zip(range(3), (D.nx, D.ny, D.nz)):
        ua = D.dirs[m, a] if a < D.dim else 0.0
        rng.append(range(n) if ua >= 0 else range(n - 1, -1, -1))
    for k in rng[2]:
        for j in rng[1]:
            for i in rng[0]:
                yield i, j, k


def sweep(D, src, sigma):
    """Solve sum_a |u_a|/h (psi_c - psi_upwind) + sigma_c psi_c = src_c per direction."""
    src = np.asarray(src, float).reshape(D.N, D.nz, D.ny, D.nx)
    sig = np.asarray(sigma, float).reshape(D.nz, D.ny, D.nx)
    psi = np.zeros_like(src)
    for m in range(D.N):
        coef = [abs(D.dirs[m, a]) / D.h if a < D.dim else 0.0 for a in range(3)]
        step = [1 if (a < D.dim and D.dirs[m, a] >= 0) else -1 for a in range(3)]
        p = psi[m]
        for i, j, k in _upwind_order(D, m):
            num = src[m, k, j, i]
            den = sig[k, j, i]
            for a, (ci, cj, ck) in enumerate(((i - step[0], j, k), (i, j - step[1], k), (i, j, k - step[2]))):
                if coef[a] == 0.0:
                    continue
                den += coef[a]
                if 0 <= ci < D.nx and 0 <= cj < D.ny and 0 <= ck < D.nz:
                    num += coef[a] * p[ck, cj, ci]
            p[k, j, i] = num / den
    return psi.reshape(D.N, D.cells)


def sweep_solve(D, b=None):
    """Exact solve when sS = 0 (L is block triangular in upwind order)."""
    if np.any(D.sS != 0.0):
        raise ValueError("sweep_solve needs a purely absorbing medium")
    b = dsc.rhs(D) if b is None else b
    return sweep(D, b, D.sT)


def source_iteration(D, b=None, tol=1e-13, max_iter=10000):
    """psi <- T^{-1}(sS S psi + b), T = streaming + sT, from psi = 0."""
    b = dsc.rhs(D) if b is None else np.asarray(b).reshape(D.N, D.cells)
    psi = np.zeros((D.N, D.cells))
    for it in range(max_iter):
        src = b + D.sS[None, :] * (D.S @ psi)
        new = sweep(D, src, D.sT)
        if np.max(np.abs(new - psi)) <= tol * max(1.0, np.max(np.abs(new))):
            return new, it + 1
        psi = new
    return psi, max_iter


def isotropic_limit(D, b_inflow):
    """Scalar flux phi_0 of the eps -> 0 limit at fixed h.

    Weighting L psi = b by w_m and summing over m removes the collision term
    up to sA phi (the scattering matrix conserves sum_m w_m psi_m).  As
    eps -> 0 the collision term forces psi_m -> phi (isotropic), sA -> 0 and
    q_hat -> 0, so phi_0 solves
        sum_m w_m sum_a |u_{m,a}|/h (phi_c - phi_{c - s_a e_a}) = sum_m w_m b_{m,c}
    with zero ghosts; b_inflow holds only the inflow part of b.
    """
    cells = D.cells
    A = np.zeros((cells, cells))
    e = np.zeros(cells)
    for c in range(cells):
        e[c] = 1.0
        col = np.zeros(cells)
        f = e.reshape(D.nz, D.ny, D.nx)
        for m in range(D.N):
            for a in D.axes:
                ua = D.dirs[m, a]
                if ua == 0.0:
                    continue
                ax = D.array_axis(a) - 1
                col += D.w[m] * abs(ua) / D.h * (f - dsc.upwind_neighbour(f, ax, ua > 0)).reshape(-1)
        A[:, c] = col
        e[c] = 0.0
    rhs = D.w @ np.asarray(b_inflow).reshape(D.N, cells)
    return np.linalg.solve(A, rhs)

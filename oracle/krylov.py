"""Right-preconditioned flexible GMRES(k) in FP64 (oracle; test infrastructure).

The paper uses the trained network as a GMRES preconditioner (Sec. 3 and
Sec. 4.2).  Because a learned preconditioner need not be a fixed linear map
(it is evaluated in reduced precision on the GPU), the flexible variant is
used: the preconditioned vectors z_j are stored and the update is x += Z y.
Orthogonalisation is modified Gram-Schmidt; the small least-squares problem is
reduced with Givens rotations; the true residual is recomputed at every
restart.
"""
import math

import numpy as np


def back_substitute(R, g):
    """Solve the upper-triangular system R y = g by back substitution."""
    j = R.shape[0]
    y = np.zeros(j)
    for i in range(j - 1, -1, -1):
        y[i] = (g[i] - R[i, i + 1:j] @ y[i + 1:j]) / R[i, i]
    return y


def fgmres(apply_A, b, precond=None, restart=30, rtol=1e-8, max_iters=5000, x0=None,
           record=None):
    """Solve A x = b.  Returns (x, stats).

    apply_A, precond: callables on flat FP64 vectors (precond None = identity).
    Stops when ||b - A x||_2 <= rtol ||b||_2 at a restart, or when the
    rotated residual estimate says so inside a cycle and the recomputed true
    residual agrees, or after max_iters inner steps.  `record`, if a list,
    receives (V, Z, Hbar, j) of every cycle for identity checks.
    """
    b = np.asarray(b, float).reshape(-1)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, float).reshape(-1)
    M = (lambda v: v) if precond is None else precond
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), dict(iterations=0, restarts=0, converged=True, rel_residual=0.0)
    r = b - apply_A(x)
    beta = np.linalg.norm(r)
    iters = 0
    restarts = 0
    k = restart
    while beta > rtol * bnorm and iters < max_iters:
        V = np.zeros((k + 1, n))
        Z = np.zeros((k, n))
        H = np.zeros((k + 1, k))
        Hraw = np.zeros((k + 1, k))
        cs = np.zeros(k)
        sn = np.zeros(k)
        g = np.zeros(k + 1)
        g[0] = beta
        V[0] = r / beta
        j_used = 0
        for j in range(k):
            Z[j] = M(V[j])
            w = apply_A(Z[j])
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            hnext = np.linalg.norm(w)
            H[j + 1, j] = hnext
            Hraw[:, j] = H[:, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rho = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / rho
            sn[j] = H[j + 1, j] / rho
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            iters += 1
            j_used = j + 1
            if hnext == 0.0:
                break
            V[j + 1] = w / hnext
            if abs(g[j + 1]) <= rtol * bnorm or iters >= max_iters:
                break
        y = back_substitute(H[:j_used, :j_used], g[:j_used])
        x = x + Z[:j_used].T @ y
        if record is not None:
            record.append((V[:j_used + 1].copy(), Z[:j_used].copy(), Hraw[:j_used + 1, :j_used].copy(), j_used))
        r = b - apply_A(x)
        beta_new = np.linalg.norm(r)
        restarts += 1
        if beta_new >= beta:            # no progress over a whole cycle
            beta = beta_new
            break
        beta = beta_new
    return x, dict(iterations=iters, restarts=restarts, converged=bool(beta <= rtol * bnorm),
                   rel_residual=float(beta / bnorm))

"""Comparator preconditioners of the oracle (test infrastructure: only tests,
the smoke check and the benchmark's CPU baseline use it).

Cell-wise Block-Jacobi: the preconditioner keeps, for every cell c, the
N x N block of L that couples the directions of that cell and drops the
couplings between cells (the upwind neighbour terms of the streaming
operator).  From the discrete operator of Sec. 2.1 (eq. (DORTE_2d) and its
3D analogue) the block is

    B_c = diag_m( sum_a |u_{m,a}| / h ) + sT_c I - sS_c S,

with sT = sigma_T / eps and sS = sigma_T / eps - eps sigma_a (the diffusive
scaling of eq. (RTE)) and S the normalised scattering matrix.  Applying the
preconditioner solves B_c z_c = v_c cell by cell.  The paper compares its
MgNet preconditioner against this one (Sec. 4, the diffusive test).
"""
import numpy as np


def cell_blocks(D):
    """B_c for every cell, shape [cells, N, N] (written from the formula above)."""
    stream = np.abs(D.dirs[:, :D.dim]).sum(axis=1) / D.h           # [N]
    B = -D.sS[:, None, None] * D.S[None, :, :]
    idx = np.arange(D.N)
    B[:, idx, idx] += stream[None, :] + D.sT[:, None]
    return B


def block_jacobi(D, v):
    """z with B_c z_c = v_c in every cell; v and z of shape [N, cells] (FP64)."""
    V = np.asarray(v, float).reshape(D.N, D.cells).T[:, :, None]      # [cells, N, 1]
    z = np.linalg.solve(cell_blocks(D), V)[:, :, 0]
    return z.T.copy()

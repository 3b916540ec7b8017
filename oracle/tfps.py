"""The tailored finite point scheme (TFPS) of Sec. 2.2, 2D, in FP64 (oracle; test infrastructure).

Only tests/, the smoke check and the benchmark's CPU baseline use this module.

In each cell C the coefficients are constant (the diffusively scaled sT, sS, q_hat
of eq. (RTE); sA = sT - sS must not vanish, as Sec. 2.2 assumes), and the local
homogeneous equation, eq. (discretization_2D_TFPS_local_homo), has the
exponential solutions of eq. (2D_eigenfunc_pre): psi = l exp(sT (xi_x x + xi_y y))
with [(sS/sT) S - I] l = (xi_x Cx + xi_y Cy) l, eq.
(discretization_2D_eigenfunc_constraint), where S = K W is the scattering matrix
and Cx, Cy are the diagonal matrices of the directions' x and y components.

Basis (eq. (2D_eigenfunc)): the N eigenpairs with xi_y = 0 and the N with
xi_x = 0, 2N functions chi^k(z) = l^k exp(sT xi^k . (z - z^k)) per cell,
||l^k||_inf = 1, each referred to the cell edge from which it decays (left edge
for xi_x < 0, right edge for xi_x > 0, bottom for xi_y < 0, top for xi_y > 0),
so |chi^k| <= 1 inside the cell.  Local order of the 2N functions (reading of
the garbled index ranges of the paper): x-type with xi_x < 0 in ascending
order, x-type with xi_x > 0 ascending, y-type with xi_y < 0 ascending, y-type
with xi_y > 0 ascending.  Particular solution chi^s = q_hat / sA (eq.
(2DTFPS_sol)).

Unknowns: the coefficients alpha, laid out [2N][ny][nx] (basis index major,
cells x fastest).  Equations, laid out [2][N][ny][nx]:
  block 0, x faces: row (m, j, i), i >= 1: continuity of psi_m at the midpoint
    of the face between cells (i-1, j) and (i, j), eq. (2DTFPS_continuity_cond),
    written psi_left - psi_right = chi^s_right - chi^s_left;
    row (m, j, 0): the inflow condition of eq. (2DTFPS_boundary_cond) at the x = 0
    face of cell (0, j) when c_m > 0, at the x = 1 face of cell (I-1, j) when
    c_m < 0 (each boundary face supplies its incoming half);
  block 1, y faces: the same along y with s_m.
The system has 2 N I^2 equations and unknowns.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import discretisation as dsc


def _sorted_eigs(M):
    """Eigenpairs of M (real spectrum) in ascending order of the eigenvalue; each vector
    scaled to max-norm 1 (the paper's normalisation), its sign fixed by making positive the
    first entry whose magnitude is within 1e-8 of the largest (symmetric direction sets give
    vectors whose largest entries tie in magnitude)."""
    w, V = np.linalg.eig(M)
    if np.max(np.abs(w.imag)) > 1e-9 * max(1.0, np.max(np.abs(w.real))):
        raise ValueError("complex eigenvalues: the cell's medium is outside the scheme's assumptions")
    w, V = w.real, V.real
    order = np.argsort(w)
    w, V = w[order], V[:, order]
    for k in range(V.shape[1]):
        a = np.abs(V[:, k])
        i = int(np.nonzero(a >= (1.0 - 1e-8) * a.max())[0][0])
        V[:, k] *= np.sign(V[i, k]) / a.max()
    return w, V


class TFPS:
    """TFPS discretisation of a 2D problem dict (the same dicts the upwind oracle takes)."""

    def __init__(self, prob):
        D = dsc.Discretisation(prob)
        if D.dim != 2:
            raise ValueError("TFPS is implemented in 2D")
        self.D = D
        N, I = D.N, D.nx
        if D.ny != I:
            raise ValueError("square grids only")
        self.N, self.I, self.h = N, I, D.h
        c, s = D.dirs[:, 0], D.dirs[:, 1]
        if np.any(c == 0) or np.any(s == 0):
            raise ValueError("directions need nonzero x and y components")
        if np.sum(c > 0) * 2 != N or np.sum(s > 0) * 2 != N:
            raise ValueError("half of the directions must point each way along x and along y")
        self.c, self.s = c, s
        # sigma_T - sigma_s of the cell in the scaled equation, taken as eps sigma_a (the
        # difference of the two scaled coefficients cancels when eps is small)
        sA = D.sA
        if np.any(sA <= 0):
            raise ValueError("TFPS needs sigma_T - sigma_s > 0 in every cell")
        self.sA = sA
        cells = D.cells
        # per cell: xi [2N], L [N, 2N]
        self.xi = np.zeros((cells, 2 * N))
        self.L = np.zeros((cells, N, 2 * N))
        cache = {}
        for cidx in range(cells):
            ratio = D.sS[cidx] / D.sT[cidx]
            if ratio not in cache:
                B = ratio * D.S - np.eye(N)
                wx, Vx = _sorted_eigs(B / c[:, None])
                wy, Vy = _sorted_eigs(B / s[:, None])
                if np.sum(wx < 0) * 2 != N or np.sum(wy < 0) * 2 != N:
                    raise ValueError("eigenvalues do not split evenly by sign")
                cache[ratio] = (np.concatenate([wx, wy]), np.concatenate([Vx, Vy], axis=1))
            self.xi[cidx], self.L[cidx] = cache[ratio]
        self.chis = D.qh / sA                        # particular solution per cell
        # exponential factor of every basis function at the four face midpoints and the centre
        self.e = {f: np.zeros((cells, 2 * N)) for f in ("left", "right", "bottom", "top", "centre")}
        h = self.h
        for cidx in range(cells):
            a = D.sT[cidx] * self.xi[cidx] * h    # sT xi h per basis function
            for k in range(2 * N):
                xtype = k < N
                neg = (k % N) < N // 2
                # position, in units of h along the function's axis, of the lower and the
                # upper face relative to the reference edge; the centre and the two faces
                # across the other axis sit half way between them
                lo_pos, hi_pos = (0.0, 1.0) if neg else (-1.0, 0.0)
                lo, hi = np.exp(a[k] * lo_pos), np.exp(a[k] * hi_pos)
                mid = np.exp(a[k] * 0.5 * (lo_pos + hi_pos))
                if xtype:
                    self.e["left"][cidx, k], self.e["right"][cidx, k] = lo, hi
                    self.e["bottom"][cidx, k] = self.e["top"][cidx, k] = mid
                else:
                    self.e["bottom"][cidx, k], self.e["top"][cidx, k] = lo, hi
                    self.e["left"][cidx, k] = self.e["right"][cidx, k] = mid
                self.e["centre"][cidx, k] = mid
        self.n = 2 * N * cells

    # ------------------------------------------------------------- values ---
    def cell(self, i, j):
        return j * self.I + i

    def face_values(self, alpha, face):
        """psi (without the particular solution) of every cell at one face midpoint: [N, cells]."""
        a = np.asarray(alpha, float).reshape(2 * self.N, -1)
        w = self.e[face].T * a                           # [2N, cells]
        return np.einsum("cmk,kc->mc", self.L, w)

    def basis_at(self, cidx, z):
        """chi^k(z) for every k of cell cidx at a point z = (x, y) (for checks): [N, 2N]."""
        I = self.I
        i, j = cidx % I, cidx // I
        h = self.h
        xl, xr, yb, yt = i * h, (i + 1) * h, j * h, (j + 1) * h
        xc, yc = xl + h / 2, yb + h / 2
        N = self.N
        out = np.zeros((N, 2 * N))
        sT = self.D.sT[cidx]
        for k in range(2 * N):
            xi = self.xi[cidx, k]
            neg = (k % N) < N // 2
            if k < N:
                zr = (xl if neg else xr, yc)
                arg = sT * xi * (z[0] - zr[0])
            else:
                zr = (xc, yb if neg else yt)
                arg = sT * xi * (z[1] - zr[1])
            out[:, k] = self.L[cidx, :, k] * np.exp(arg)
        return out

    def psi_centres(self, alpha):
        """psi_m at every cell centre, [N, cells] (eq. (2DTFPS_sol) evaluated at the centres)."""
        return self.face_values(alpha, "centre") + self.chis[None, :]

    # ------------------------------------------------------------ system ---
    def apply(self, alpha):
        """y = A alpha in the equation layout [2, N, ny, nx] (flattened)."""
        N, I = self.N, self.I
        L_ = self.face_values(alpha, "left").reshape(N, I, I)
        R_ = self.face_values(alpha, "right").reshape(N, I, I)
        B_ = self.face_values(alpha, "bottom").reshape(N, I, I)
        T_ = self.face_values(alpha, "top").reshape(N, I, I)
        y = np.zeros((2, N, I, I))
        # x faces: interior i >= 1 -> psi of cell (i-1) at its right face minus psi of cell i at its left face
        y[0, :, :, 1:] = R_[:, :, :-1] - L_[:, :, 1:]
        cpos = self.c > 0
        y[0, cpos, :, 0] = L_[cpos, :, 0]
        y[0, ~cpos, :, 0] = R_[~cpos, :, I - 1]
        y[1, :, 1:, :] = T_[:, :-1, :] - B_[:, 1:, :]
        spos = self.s > 0
        y[1, spos, 0, :] = B_[spos, 0, :]
        y[1, ~spos, 0, :] = T_[~spos, I - 1, :]
        return y.reshape(-1)

    def rhs(self):
        """b: jumps of the particular solutions across interior faces and the inflow data
        minus the particular solution at boundary faces."""
        D, N, I = self.D, self.N, self.I
        cs = self.chis.reshape(I, I)
        b = np.zeros((2, N, I, I))
        b[0, :, :, 1:] = (cs[:, 1:] - cs[:, :-1])[None]
        b[1, :, 1:, :] = (cs[1:, :] - cs[:-1, :])[None]
        def inflow(face, m):
            v = dsc.face_values(D, face, m)
            return np.zeros(I) if v is None else v.reshape(-1)[:I]
        for m in range(N):
            if self.c[m] > 0:
                b[0, m, :, 0] = inflow(0, m) - cs[:, 0]
            else:
                b[0, m, :, 0] = inflow(1, m) - cs[:, I - 1]
            if self.s[m] > 0:
                b[1, m, 0, :] = inflow(2, m) - cs[0, :]
            else:
                b[1, m, 0, :] = inflow(3, m) - cs[I - 1, :]
        return b.reshape(-1)

    def assemble(self):
        """A as a sparse matrix, column by column from the definition of each equation."""
        N, I = self.N, self.I
        rows, cols, vals = [], [], []

        def eq(blk, m, j, i):
            return ((blk * N + m) * I + j) * I + i

        def unk(k, cidx):
            return k * I * I + cidx

        for j in range(I):
            for i in range(I):
                cidx = self.cell(i, j)
                V = {f: self.L[cidx] * self.e[f][cidx][None, :] for f in ("left", "right", "bottom", "top")}
                for m in range(N):
                    targets = []
                    # this cell's left face: row (0, m, j, i) with sign -1 (i >= 1) or the inflow row
                    if i >= 1:
                        targets.append((eq(0, m, j, i), -1.0, "left"))
                    elif self.c[m] > 0:
                        targets.append((eq(0, m, j, 0), 1.0, "left"))
                    if i + 1 < I:
                        targets.append((eq(0, m, j, i + 1), 1.0, "right"))
                    elif self.c[m] < 0:
                        targets.append((eq(0, m, j, 0), 1.0, "right"))
                    if j >= 1:
                        targets.append((eq(1, m, j, i), -1.0, "bottom"))
                    elif self.s[m] > 0:
                        targets.append((eq(1, m, 0, i), 1.0, "bottom"))
                    if j + 1 < I:
                        targets.append((eq(1, m, j + 1, i), 1.0, "top"))
                    elif self.s[m] < 0:
                        targets.append((eq(1, m, 0, i), 1.0, "top"))
                    for r, sgn, f in targets:
                        for k in range(2 * N):
                            rows.append(r)
                            cols.append(unk(k, cidx))
                            vals.append(sgn * V[f][m, k])
        return sp.csr_matrix((vals, (rows, cols)), shape=(self.n, self.n))

    def solve(self):
        """alpha solving A alpha = b (sparse LU)."""
        A = self.assemble().tocsc()
        return spla.spsolve(A, self.rhs())

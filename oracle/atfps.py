"""The adaptive tailored finite point scheme (ATFPS) of Sec. 2.3, 2D, in FP64 (oracle; test infrastructure).

Only tests/, the smoke check and the benchmark's CPU baseline use this module.

Built on the TFPS discretisation of oracle.tfps (same per-cell bases, same local order:
functions centred at the left, right, bottom and top face of the cell, N/2 each).

1. Selection, eq. (def_V_delta): cell C keeps basis function k when its value at the cell
   centre, exp(-|xi_k| sT h / 2), exceeds delta; the rest are the fast-decaying (layer)
   functions.
2. Interface bases: for each face, the functions centred on it (from the one or two cells
   that share it).  The kept ones' eigenvectors are orthonormalised by a QR factorisation;
   the dropped ones' eigenvectors follow as they are; every vector is scaled to max-norm 1
   (reading: the orthonormalised ones with the sign rule of the eigenvectors, since the QR
   factors are unique only up to column signs).
   On a boundary face only the incoming directions enter.  P^k is the coefficient of a
   vector on the k-th vector of that basis.
3. Compressed system, eq. (2DAdaptiveTFPS_linear_sys): unknowns are the kept coefficients;
   for every face and every kept function centred on it, the projection of the TFPS
   continuity condition (eq. (2DAdaptiveTFPS_continuity_cond)) or inflow condition
   (eq. (2DAdaptiveTFPS_boundary_cond)) onto that basis vector, with the kept functions of
   both cells (the dropped ones are neglected, an O(delta) error).
4. Layer reconstruction, eq. (2DAdaptive_TFPS_layer1) and (2DAdaptive_TFPS_layer2): each
   dropped coefficient is the projection of the jump of the smooth solution (or of the
   inflow data minus the smooth solution) across its face onto its own basis vector.
5. The filtered loss of Sec. 3.4, eq. (loss_delta): || b_delta - A_delta D_delta psi_d ||_2,
   with D_delta the per-cell least-squares map from cell-centre values to kept coefficients
   (reading: the paper does not define D; this is the minimum-norm least-squares fit of the
   cell-centre values minus the particular solution by the kept functions, singular values
   at or below machine epsilon times max(N, kept) times the largest taken as zero, so that
   kept functions which coincide at the centre give the minimum-norm fit).

Row order of the compressed system: x faces (faces x_i, i = 0..I, for each grid row j,
i fastest), then y faces (faces y_j, j = 0..I, for each grid column i, j fastest); within
a face its kept basis vectors in order.  Unknown order: cell by cell (x fastest), the
kept indices of each cell ascending.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import discretisation as dsc
from .tfps import TFPS

FACES = ("left", "right", "bottom", "top")


def _centred_on(k, N):
    """Face on which local basis function k of a cell is centred (0 left, 1 right, 2 bottom, 3 top)."""
    return k // (N // 2)


def _maxnorm(V):
    big = np.max(np.abs(V), axis=0)
    return V / big[None, :]


def _maxnorm_signed(V):
    """Columns scaled to max-norm 1, each with its first entry within 1e-8 of the largest
    magnitude positive (the QR factors are unique up to the signs of their columns)."""
    out = np.array(V, float)
    for k in range(out.shape[1]):
        a = np.abs(out[:, k])
        i = int(np.nonzero(a >= (1.0 - 1e-8) * a.max())[0][0])
        out[:, k] *= np.sign(out[i, k]) / a.max()
    return out


class ATFPS:
    def __init__(self, prob, delta):
        self.T = T = TFPS(prob)
        self.delta = float(delta)
        D, N, I = T.D, T.N, T.I
        self.N, self.I = N, I
        cells = I * I
        self.cells = cells
        # 1. selection
        self.keep = np.exp(-0.5 * np.abs(T.xi) * D.sT[:, None] * T.h) > self.delta   # [cells, 2N]
        self.kidx = [np.nonzero(self.keep[c])[0] for c in range(cells)]
        self.offset = np.concatenate([[0], np.cumsum([len(k) for k in self.kidx])])
        self.n = int(self.offset[-1])
        # 2. faces: (cells with their local functions centred here, direction mask, basis)
        self.faces = []
        c_in = T.c > 0
        s_in = T.s > 0
        for j in range(I):                    # x faces, x_i for i = 0..I
            for i in range(I + 1):
                parts = []
                if i >= 1:
                    parts.append((T.cell(i - 1, j), 1, -1.0))   # left cell, its right-centred functions
                if i < I:
                    parts.append((T.cell(i, j), 0, +1.0))       # right cell, its left-centred functions
                mask = None if len(parts) == 2 else (c_in if i == 0 else ~c_in)
                self.faces.append(self._face(parts, mask, "x", (i, j)))
        for i in range(I):                    # y faces, y_j for j = 0..I
            for j in range(I + 1):
                parts = []
                if j >= 1:
                    parts.append((T.cell(i, j - 1), 3, -1.0))
                if j < I:
                    parts.append((T.cell(i, j), 2, +1.0))
                mask = None if len(parts) == 2 else (s_in if j == 0 else ~s_in)
                self.faces.append(self._face(parts, mask, "y", (i, j)))

    def _face(self, parts, mask, axis, pos):
        """One face: the functions centred on it, its basis H (columns: kept ones orthonormalised
        then dropped ones), and the face-value operators of the cells on each side."""
        T, N = self.T, self.N
        rows = np.arange(N) if mask is None else np.nonzero(mask)[0]
        kept, dropped = [], []
        for cidx, fc, sign in parts:
            for k in range(fc * (N // 2), (fc + 1) * (N // 2)):
                (kept if self.keep[cidx, k] else dropped).append((cidx, k))
        Lk = np.array([T.L[c][rows, k] for c, k in kept]).T.reshape(len(rows), len(kept))
        Ld = np.array([T.L[c][rows, k] for c, k in dropped]).T.reshape(len(rows), len(dropped))
        if len(kept):
            Q, _ = np.linalg.qr(Lk)
            Q = _maxnorm_signed(Q)
        else:
            Q = np.zeros((len(rows), 0))
        H = np.concatenate([Q, _maxnorm(Ld) if len(dropped) else Ld], axis=1)
        if H.shape[1] != len(rows):
            raise ValueError("face basis does not span the face's directions")
        Hinv = np.linalg.inv(H)
        # which face of each side's cell this face is (for the exponential factors)
        side = []
        for cidx, fc, sign in parts:
            side.append((cidx, FACES[fc], sign))
        return dict(axis=axis, pos=pos, rows=rows, kept=kept, dropped=dropped, Hinv=Hinv, side=side,
                    nkeep=len(kept), boundary=mask is not None)

    # --------------------------------------------------------------- values ---
    def face_vector(self, cidx, face, coef, which):
        """psi (no particular solution) of cell cidx at a face midpoint, from its coefficients
        restricted to `which` ('kept', 'all' or an explicit index array)."""
        T = self.T
        a = np.zeros(2 * self.N)
        if which == "kept":
            a[self.kidx[cidx]] = coef[self.kidx[cidx]]
        else:
            a[:] = coef
        return T.L[cidx] @ (T.e[face][cidx] * a)

    def scatter(self, alpha):
        """Compressed unknowns -> full per-cell coefficient array [cells, 2N] (dropped ones 0)."""
        full = np.zeros((self.cells, 2 * self.N))
        for c in range(self.cells):
            full[c, self.kidx[c]] = alpha[self.offset[c]:self.offset[c + 1]]
        return full

    # --------------------------------------------------------------- system ---
    def assemble(self):
        """(A_delta, b_delta) of eq. (2DAdaptiveTFPS_linear_sys), row by row from the
        projected conditions."""
        T, N = self.T, self.N
        rows, cols, vals, b = [], [], [], []
        r = 0
        D = T.D
        for f in self.faces:
            P = f["Hinv"][:f["nkeep"]]                 # projections onto the kept basis vectors
            rhs = np.zeros(len(f["rows"]))
            for cidx, face, sign in f["side"]:
                # sign +1: the cell right of / above the face (moves to the right side of the
                # continuity condition); boundary faces have a single cell with sign +1
                s_eq = 1.0 if f["boundary"] else -sign
                E = (T.L[cidx] * T.e[face][cidx][None, :])[f["rows"]]      # [rows, 2N]
                for q, k in enumerate(self.kidx[cidx]):
                    col = self.offset[cidx] + q
                    v = P @ E[:, k]
                    for p in range(f["nkeep"]):
                        rows.append(r + p)
                        cols.append(col)
                        vals.append(s_eq * v[p])
                rhs -= s_eq * T.chis[cidx]
            if f["boundary"]:
                rhs += self._inflow(f)
            b.append(P @ rhs)
            r += f["nkeep"]
        A = sp.csr_matrix((vals, (rows, cols)), shape=(r, self.n))
        return A, np.concatenate(b) if b else np.zeros(0)

    def _inflow(self, f):
        D, I = self.T.D, self.I
        i, j = f["pos"]
        if f["axis"] == "x":
            face, idx = (0 if i == 0 else 1), j
        else:
            face, idx = (2 if j == 0 else 3), i
        out = np.zeros(len(f["rows"]))
        for q, m in enumerate(f["rows"]):
            v = dsc.face_values(D, face, m)
            out[q] = 0.0 if v is None else v.reshape(-1)[idx]
        return out

    def solve(self):
        """Kept coefficients alpha_delta (sparse LU of the compressed system)."""
        A, b = self.assemble()
        if A.shape[0] != A.shape[1]:
            raise ValueError("compressed system is not square")
        return spla.spsolve(A.tocsc(), b)

    # -------------------------------------------------------- reconstruction ---
    def reconstruct(self, alpha):
        """All coefficients [cells, 2N]: the kept ones, and the dropped ones from eq.
        (2DAdaptive_TFPS_layer1) / (2DAdaptive_TFPS_layer2)."""
        T = self.T
        full = self.scatter(alpha)
        smooth = self.scatter(alpha)
        for f in self.faces:
            if not f["dropped"]:
                continue
            Pd = f["Hinv"][f["nkeep"]:]              # projections onto the dropped basis vectors
            vals = {}
            for cidx, face, sign in f["side"]:
                vals[cidx] = (self.face_vector(cidx, face, smooth[cidx], "all") + T.chis[cidx])[f["rows"]]
            if f["boundary"]:
                (cidx, face, sign), = f["side"]
                proj = Pd @ (self._inflow(f) - vals[cidx])
                for q, (c, k) in enumerate(f["dropped"]):
                    full[c, k] = proj[q]
            else:
                (cm, _, _), (cp, _, _) = f["side"]
                proj_m, proj_p = Pd @ vals[cm], Pd @ vals[cp]
                for q, (c, k) in enumerate(f["dropped"]):
                    full[c, k] = (proj_p[q] - proj_m[q]) if c == cm else (proj_m[q] - proj_p[q])
        return full

    def psi_centres(self, full):
        """psi at the cell centres from a full coefficient array [cells, 2N] (as oracle.tfps)."""
        return self.T.psi_centres(np.asarray(full).T.reshape(-1))

    # ---------------------------------------------------------- filtered loss ---
    def D_map(self, psi_centres):
        """Kept coefficients from cell-centre values [N, cells]: per cell the minimum-norm
        least-squares fit of psi - chi^s by the kept functions at the centre (the SVD cutoff
        is numpy's default, machine epsilon times the larger dimension)."""
        T = self.T
        out = np.zeros(self.n)
        for c in range(self.cells):
            k = self.kidx[c]
            if len(k) == 0:
                continue
            M = T.L[c][:, k] * T.e["centre"][c][k][None, :]
            sol, *_ = np.linalg.lstsq(M, psi_centres[:, c] - T.chis[c], rcond=None)
            out[self.offset[c]:self.offset[c + 1]] = sol
        return out

    def filtered_loss(self, psi_centres, A=None, b=None):
        """|| b_delta - A_delta D_delta psi ||_2 of eq. (loss_delta)."""
        if A is None:
            A, b = self.assemble()
        return float(np.linalg.norm(b - A @ self.D_map(psi_centres)))

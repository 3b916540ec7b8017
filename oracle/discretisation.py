"""Setup and the discrete transport operator, in FP64 (oracle; test infrastructure).

Continuous problem: the steady RTE under diffusive scaling, eq. (RTE) of
Sec. 1, with the Henyey-Greenstein kernel of eq. (hg), inflow Dirichlet data
on Gamma^- (eq. (boundary_condition)) and interface continuity.  Angles are
discretised by discrete ordinates (Sec. 2.1, eq. (DORTE_2d)); coefficients are
constant per cell (Sec. 2.2).  Space is discretised by the cell-centred
first-order upwind finite-volume scheme:

  (L psi)_{m,c} = sum_a |u_{m,a}|/h (psi_{m,c} - psi_{m,c - s_a e_a})
                  + sT_c psi_{m,c} - sS_c sum_n S_{mn} psi_{n,c}

with s_a = sign(u_{m,a}), out-of-domain neighbours zero (their inflow data sit
in the right-hand side), sT = sigma_T/eps, sS = sigma_T/eps - eps sigma_a and
S = K W the quadrature-weighted, symmetrically normalised kernel matrix.

Arrays: psi has shape [N, cells] with cells ordered x fastest; internally it
is viewed as [N, nz, ny, nx].
"""
import numpy as np


# ----------------------------------------------------------------- kernel ---

def kernel_kind(dirs, kind):
    """'flatland' for circle sets, 'sphere' otherwise, unless given explicitly."""
    if kind in ("flatland", "sphere"):
        return kind
    return "flatland" if np.all(dirs[:, 2] == 0.0) else "sphere"


def hg_matrix(dirs, g, kind):
    """Unnormalised kernel values P_mn = kappa(u_m . u_n).

    'sphere' is eq. (hg) as printed: (1 - g^2) / (1 + g^2 - 2 g mu)^(3/2).
    'flatland' is its two-dimensional analogue (1 - g^2) / (1 + g^2 - 2 g mu),
    whose mean cosine on the circle is g.
    """
    mu = np.clip(dirs @ dirs.T, -1.0, 1.0)
    base = 1.0 + g * g - 2.0 * g * mu
    if kind == "sphere":
        return (1.0 - g * g) / base ** 1.5
    return (1.0 - g * g) / base


def symmetric_scaling(P, w, tol=1e-15, max_iter=100000):
    """Positive d with sum_n d_m P_mn d_n w_n = 1 for every m.

    Iterates d <- sqrt(d / (P W d)); the fixed point makes D P D a symmetric
    matrix whose w-weighted rows (and, by symmetry, columns) sum to one.
    """
    d = np.ones(P.shape[0])
    for _ in range(max_iter):
        d_new = np.sqrt(d / (P @ (w * d)))
        if np.max(np.abs(d_new - d)) <= tol * np.max(d_new):
            d = d_new
            break
        d = d_new
    return d


def scatter_matrix(dirs, w, g, kind="auto"):
    """S = K W with K = D P D (Sec. 2.1: kappa_mn approximates the kernel).

    Returns (S, K).  (S psi)_m = sum_n K_mn w_n psi_n.
    """
    kind = kernel_kind(dirs, kind)
    P = hg_matrix(dirs, g, kind)
    d = symmetric_scaling(P, w)
    K = d[:, None] * P * d[None, :]
    return K * w[None, :], K


# ---------------------------------------------------------------- problem ---

class Discretisation:
    """All arrays the operator and right-hand side need, built from a problem dict."""

    def __init__(self, prob):
        self.dim = prob["dim"]
        self.nx, self.ny, self.nz = prob["n"]
        self.cells = self.nx * self.ny * self.nz
        self.h = 1.0 / self.nx
        self.dirs = np.asarray(prob["dirs"], float)
        self.w = np.asarray(prob["weights"], float)
        self.N = self.dirs.shape[0]
        self.n = self.N * self.cells
        self.g = prob["g"]
        self.kind = kernel_kind(self.dirs, prob.get("kernel", "auto"))
        self.S, self.K = scatter_matrix(self.dirs, self.w, self.g, self.kind)
        st = np.asarray(prob["sigma_t"], float).reshape(-1)
        sa = np.asarray(prob["sigma_a"], float).reshape(-1)
        q = np.asarray(prob["q"], float).reshape(-1)
        eps = prob["eps"]
        eps = np.full(self.cells, float(eps)) if np.isscalar(eps) else np.asarray(eps, float).reshape(-1)
        # diffusive scaling of eq. (RTE)
        self.sigma_t, self.sigma_a, self.q, self.eps = st, sa, q, eps
        self.sT = st / eps
        self.sS = st / eps - eps * sa
        self.sA = eps * sa
        self.qh = eps * q
        self.inflow = prob.get("inflow")
        self.axes = [a for a in range(self.dim)]

    # shape helpers
    def grid(self, v):
        return np.asarray(v).reshape(-1, self.nz, self.ny, self.nx)

    def flat(self, v):
        return np.asarray(v).reshape(self.N, self.cells)

    @staticmethod
    def array_axis(a):
        return 3 - a            # x -> last axis, y -> axis 2, z -> axis 1


def upwind_neighbour(f, axis, positive):
    """Values at c - s e_a along `axis` of a [nz, ny, nx] array, zero outside."""
    g = np.zeros_like(f)
    src = [slice(None)] * f.ndim
    dst = [slice(None)] * f.ndim
    if positive:
        dst[axis] = slice(1, None)
        src[axis] = slice(None, -1)
    else:
        dst[axis] = slice(None, -1)
        src[axis] = slice(1, None)
    g[tuple(dst)] = f[tuple(src)]
    return g


def apply_L(D, psi):
    """y = L psi for psi of shape [N, cells] (or anything reshapeable to it)."""
    x = D.grid(psi)
    y = np.zeros_like(x)
    for m in range(D.N):
        for a in D.axes:
            ua = D.dirs[m, a]
            if ua == 0.0:
                continue
            ax = D.array_axis(a) - 1
            y[m] += abs(ua) / D.h * (x[m] - upwind_neighbour(x[m], ax, ua > 0))
    Sx = np.tensordot(D.S, x, axes=(1, 0))
    sT = D.sT.reshape(D.nz, D.ny, D.nx)
    sS = D.sS.reshape(D.nz, D.ny, D.nx)
    y += sT[None] * x - sS[None] * Sx
    return y.reshape(D.N, D.cells)


def diagonal(D):
    """Diagonal of L: sum_a |u_{m,a}|/h + sT_c - sS_c S_mm, shape [N, cells]."""
    stream = np.abs(D.dirs[:, :D.dim]).sum(axis=1) / D.h
    return stream[:, None] + D.sT[None, :] - D.sS[None, :] * np.diag(D.S)[:, None]


def face_values(D, face, m):
    """Inflow data of face `face` for direction m as a 2D array over the face."""
    if D.inflow is None:
        return None
    axis = face // 2
    shape = {0: (D.nz, D.ny), 1: (D.nz, D.nx), 2: (D.ny, D.nx)}[axis]
    cnt = shape[0] * shape[1]
    return np.asarray(D.inflow[face, m, :cnt], float).reshape(shape)


def rhs(D):
    """b = q_hat plus the inflow carried across each boundary face (eq. (boundary_condition_2d)).

    For a cell whose upwind face along axis a is on the boundary, the face
    flux |u_{m,a}|/h * Psi_m(face midpoint) moves to the right-hand side.
    """
    b = np.tile(D.qh.reshape(1, D.nz, D.ny, D.nx), (D.N, 1, 1, 1)).astype(float)
    if D.inflow is None:
        return b.reshape(D.N, D.cells)
    for m in range(D.N):
        for a in D.axes:
            ua = D.dirs[m, a]
            if ua == 0.0:
                continue
            face = 2 * a + (0 if ua > 0 else 1)     # x- face feeds u_x > 0
            vals = face_values(D, face, m)
            coef = abs(ua) / D.h
            idx = 0 if ua > 0 else -1
            if a == 0:
                b[m, :, :, idx] += coef * vals
            elif a == 1:
                b[m, :, idx, :] += coef * vals
            else:
                b[m, idx, :, :] += coef * vals
    return b.reshape(D.N, D.cells)


def residual(D, psi, b=None):
    """r = b - L psi."""
    if b is None:
        b = rhs(D)
    return b - apply_L(D, psi)


def scalar_flux(D, psi):
    """phi_c = sum_m w_m psi_{m,c}."""
    return D.w @ D.flat(psi)

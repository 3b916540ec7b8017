"""Pins of the oracle's multi-level V-cycle composition (Sec. 3.3).

The oracle's V-cycle is a recursion over levels of smoothing steps,
restriction of the residual, a coarse solve and prolongation.  Its order --
which smoother weights act before and after the coarse correction, which field
is restricted, how many steps run on each level -- is checked here against two
independent routes:

1. a closed form.  With A = 0, a^[l] = alpha_l and a^{-1,[l]} = gamma_l
   constant, B_{l,i} = beta_{l,i} times the identity on the tap that reads the
   right-hand neighbour (the shift S: (S x)(i, j) = x(i, j + 1), zero past the
   edge), a centre-tap restriction (injection of the even pixels followed by a
   channel matrix) and a single-tap transposed convolution (the coarse value
   placed on the even fine pixel through a channel matrix), each smoothing
   step is u <- u + beta gamma S (f - alpha u), and the transfers are plain
   array slices.  The residual after the pre-smoothing steps is
   prod_i (I - alpha gamma beta_i S) f, and the coarse correction (injection)
   does not commute with S, so with distinct scalars on every level and step
   swapping the pre- and post-smoothing lists, restricting u instead of the
   residual, or dropping one step on any level changes the result;
2. a dense matrix product.  For a two-level network with general weights and
   fields, every convolution is assembled column by column from PyTorch's
   conv2d / conv_transpose2d, and the V-cycle is composed as products of
   those matrices in the order of the method.
"""
import numpy as np
import pytest

import problems
from oracle import network
from oracle import solve as osolve
from rte_inputs import configs, weights

T = weights.tag


def _closed_form_case(levels=3, N=4, c0=6, n=16, seed=5):
    """Problem, net and the scalars of the closed-form special case."""
    prob = problems.make(n=n, ndir=N, g=0.4, eps=0.2, seed=seed,
                         mg=dict(c0=c0, levels=levels, nu_pre=2, nu_post=2, nu_coarse=2, coef_ch=3,
                                 seed=seed + 1))
    hdr, t = configs.problem_weights(prob)
    rng = np.random.default_rng(seed + 2)
    sc = dict(alpha=[0.3 + 0.2 * l for l in range(levels)],
              gamma=[0.9 - 0.15 * l for l in range(levels)],
              pre=[[0.35 + 0.1 * l, 0.8 - 0.05 * l] for l in range(levels - 1)],
              post=[[1.1 + 0.07 * l, 0.25 + 0.02 * l] for l in range(levels - 1)],
              coarse=[0.6, 0.45], s=0.7,
              W_in=rng.standard_normal((c0, N)), W_out=rng.standard_normal((N, c0)),
              R=[], Pr=[])
    t[T(weights.K_WIN)][:] = sc["W_in"]
    t[T(weights.K_WOUT)][:] = sc["W_out"]
    t[T(weights.K_S)][:] = sc["s"]

    def centre(beta, C):   # beta times the identity on the tap (1, 2): reads pixel (i, j + 1)
        W = np.zeros((C, C, 3, 3))
        W[np.arange(C), np.arange(C), 1, 2] = beta
        return W

    for l in range(levels):
        C = c0 << l
        t[T(weights.K_A, l)][:] = 0
        t[T(weights.K_HAW, l)][:] = 0
        t[T(weights.K_HAB, l)][:] = sc["alpha"][l]
        t[T(weights.K_HIW, l)][:] = 0
        t[T(weights.K_HIB, l)][:] = sc["gamma"][l]
        if l < levels - 1:
            for i in range(2):
                t[T(weights.K_BPRE, l, i)][:] = centre(sc["pre"][l][i], C)
                t[T(weights.K_BPOST, l, i)][:] = centre(sc["post"][l][i], C)
            Rc = rng.standard_normal((2 * C, C)) / np.sqrt(C)
            R = np.zeros((2 * C, C, 3, 3))
            R[:, :, 1, 1] = Rc
            t[T(weights.K_R, l)][:] = R
            Pc = rng.standard_normal((2 * C, C)) / np.sqrt(2 * C)
            Pr = np.zeros((2 * C, C, 4, 4))
            Pr[:, :, 1, 1] = Pc
            t[T(weights.K_PR, l)][:] = Pr
            sc["R"].append(Rc.astype(np.float32).astype(np.float64))
            sc["Pr"].append(Pc.astype(np.float32).astype(np.float64))
        else:
            for i in range(2):
                t[T(weights.K_BC, l, i)][:] = centre(sc["coarse"][i], C)
    # the blob stores float32: the closed form uses the stored values
    for k in ("W_in", "W_out"):
        sc[k] = sc[k].astype(np.float32).astype(np.float64)
    for k in ("alpha", "gamma", "coarse"):
        sc[k] = [float(np.float32(x)) for x in sc[k]]
    for k in ("pre", "post"):
        sc[k] = [[float(np.float32(x)) for x in row] for row in sc[k]]
    sc["s"] = float(np.float32(sc["s"]))
    blob = weights.pack_mgn1(hdr, t)
    return prob, blob, sc


def _closed_form_vcycle(sc, v, diag, n, N, levels):
    """The special case's V-cycle by hand: scalar smoothing recurrences and slices."""
    vt = (v / diag).reshape(N, n, n)
    f = [None] * levels
    u = [None] * levels
    f[0] = np.einsum("cm,myx->cyx", sc["W_in"], vt)

    def shift(x):          # (S x)(i, j) = x(i, j + 1), zero past the last column
        y = np.zeros_like(x)
        y[:, :, :-1] = x[:, :, 1:]
        return y

    def smooth(l, f_l, u_l, betas):
        a, g = sc["alpha"][l], sc["gamma"][l]
        for b in betas:
            u_l = u_l + b * g * shift(f_l - a * u_l)
        return u_l

    for l in range(levels - 1):
        u[l] = smooth(l, f[l], np.zeros_like(f[l]), sc["pre"][l])
        r = f[l] - sc["alpha"][l] * u[l]
        f[l + 1] = np.einsum("dc,cyx->dyx", sc["R"][l], r[:, 0::2, 0::2])
    L1 = levels - 1
    u[L1] = smooth(L1, f[L1], np.zeros_like(f[L1]), sc["coarse"])
    for l in range(levels - 2, -1, -1):
        u[l] = u[l].copy()
        u[l][:, 0::2, 0::2] += np.einsum("dc,dyx->cyx", sc["Pr"][l], u[l + 1])
        u[l] = smooth(l, f[l], u[l], sc["post"][l])
    z = sc["s"] * vt + np.einsum("mc,cyx->myx", sc["W_out"], u[0])
    return z.reshape(N, n * n)


@pytest.mark.parametrize("levels", [2, 3, 4])
def test_vcycle_closed_form_with_scalar_smoothers(levels):
    n, N = 16, 4
    prob, blob, sc = _closed_form_case(levels=levels, N=N, n=n)
    P = osolve.Problem(prob, blob)
    rng = np.random.default_rng(7)
    for _ in range(3):
        v = rng.standard_normal((N, n * n))
        z = P.precond(v.reshape(-1)).reshape(N, n * n)
        ref = _closed_form_vcycle(sc, v, P.diag.reshape(N, -1), n, N, levels)
        assert np.max(np.abs(z - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_closed_form_scalars_separate_the_plausible_misorderings():
    """The scalars are chosen so that each plausible composition mistake moves the
    closed form itself: otherwise agreement above would not exclude it."""
    levels, n, N = 3, 16, 4
    prob, blob, sc = _closed_form_case(levels=levels, N=N, n=n)
    P = osolve.Problem(prob, blob)
    v = np.random.default_rng(8).standard_normal((N, n * n))
    d = P.diag.reshape(N, -1)
    ref = _closed_form_vcycle(sc, v, d, n, N, levels)
    swapped = dict(sc, pre=sc["post"], post=sc["pre"])
    dropped = dict(sc, post=[sc["post"][0], sc["post"][1][:1]])
    for alt in (swapped, dropped):
        z = _closed_form_vcycle(alt, v, d, n, N, levels)
        assert np.max(np.abs(z - ref)) > 1e-3 * np.max(np.abs(ref))
    # restricting u instead of the residual: (I - p(S)) f / alpha in place of p(S) f,
    # p(S) = prod_i (I - alpha gamma beta_i S); compare the two on the first level
    f0 = np.einsum("cm,myx->cyx", sc["W_in"], (v / d).reshape(N, n, n))
    a, g = sc["alpha"][0], sc["gamma"][0]
    u, r = np.zeros_like(f0), f0.copy()
    for b in sc["pre"][0]:
        sh = np.zeros_like(r)
        sh[:, :, :-1] = r[:, :, 1:]
        u = u + b * g * sh
        r = f0 - a * u
    assert np.max(np.abs(u - r)) > 0.1 * np.max(np.abs(r))


# --------------------------------------------- dense matrix composition ---

def _conv_matrix(fn, W, in_shape, **kw):
    torch = pytest.importorskip("torch")
    n_in = int(np.prod(in_shape))
    cols = []
    Wt = torch.from_numpy(np.ascontiguousarray(W))
    for j in range(n_in):
        e = np.zeros(n_in)
        e[j] = 1.0
        y = fn(torch.from_numpy(e.reshape((1,) + in_shape)), Wt, **kw)[0].numpy()
        cols.append(y.reshape(-1))
    return np.stack(cols, axis=1)


def test_two_level_vcycle_is_the_product_of_its_dense_operators():
    torch = pytest.importorskip("torch")
    F = torch.nn.functional
    n, N, c0 = 4, 4, 2
    prob = problems.make(n=n, ndir=N, g=0.3, eps=0.3, seed=11,
                         mg=dict(c0=c0, levels=2, nu_pre=2, nu_post=1, nu_coarse=2, coef_ch=3, seed=12))
    hdr, t = configs.problem_weights(prob)
    rng = np.random.default_rng(13)
    for k in list(t):   # general weights of order one everywhere (A != 0)
        t[k] = rng.standard_normal(t[k].shape).astype(np.float32) * (0.5 if (k >> 16) < 10 else 0.3)
    blob = weights.pack_mgn1(hdr, t)
    net = network.Net(blob)
    P = osolve.Problem(prob, blob)
    C0, C1, n1 = c0, 2 * c0, n // 2
    fields = ([rng.standard_normal((C0, n, n)), rng.standard_normal((C1, n1, n1))],
              [rng.standard_normal((C0, n, n)), rng.standard_normal((C1, n1, n1))])
    a, ainv = fields
    sh0, sh1 = (C0, n, n), (C1, n1, n1)
    I0, I1 = np.eye(C0 * n * n), np.eye(C1 * n1 * n1)
    conv0 = lambda W: _conv_matrix(F.conv2d, W, sh0, padding=1)
    conv1_ = lambda W: _conv_matrix(F.conv2d, W, sh1, padding=1)
    K0 = conv0(net.A[0]) + np.diag(a[0].reshape(-1))
    K1 = conv1_(net.A[1]) + np.diag(a[1].reshape(-1))
    G0, G1 = np.diag(ainv[0].reshape(-1)), np.diag(ainv[1].reshape(-1))
    Rm = _conv_matrix(F.conv2d, net.R[0], sh0, stride=2, padding=1)
    Pm = _conv_matrix(F.conv_transpose2d, net.Pr[0], sh1, stride=2, padding=1)

    def steps(U, Bs, conv, G, K, I):
        # u <- u + B Gamma (f - K u), tracked as the matrix U with u = U f
        for B in Bs:
            U = U + conv(B) @ G @ (I - K @ U)
        return U

    Dinv = np.diag(1.0 / P.diag.reshape(-1))                 # v -> v~, [N * cells]
    Win = np.kron(net.W_in, np.eye(n * n))                   # v~ -> f_0
    Wout = np.kron(net.W_out, np.eye(n * n))                 # u_0 -> z
    U0 = steps(np.zeros_like(I0), net.Bpre[0], conv0, G0, K0, I0)
    F1 = Rm @ (I0 - K0 @ U0)                                 # f_0 -> f_1 (restricted residual)
    U1 = steps(np.zeros_like(I1), net.Bc, conv1_, G1, K1, I1)
    Ufull = U0 + Pm @ U1 @ F1                                # u_0 after the coarse correction
    for B in net.Bpost[0]:
        Ufull = Ufull + conv0(B) @ G0 @ (I0 - K0 @ Ufull)
    M = net.s * Dinv + Wout @ Ufull @ Win @ Dinv
    for j in range(4):
        v = rng.standard_normal(P.D.n)
        z = network.vcycle(net, fields, P.diag, v, P.D).reshape(-1)
        ref = M @ v
        assert np.max(np.abs(z - ref)) <= 1e-12 * np.max(np.abs(ref))

"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against an independent route to the same value:
a closed form, a series expansion, a dense LU, a transport sweep, a
conservation identity, a limit, or PyTorch's convolution routines.
"""
import numpy as np
import pytest

import problems
from oracle import direct, krylov, network
from oracle import discretisation as dsc
from oracle import solve as osolve
from rte_inputs import configs, quadrature, weights


# ------------------------------------------------- kernel matrix (eq. hg) ---

def test_flatland_kernel_is_the_poisson_series():
    dirs, _ = quadrature.circle(16)
    th = np.arctan2(dirs[:, 1], dirs[:, 0])
    dth = th[:, None] - th[None, :]
    for g in (0.0, 0.3, 0.9, -0.5):
        P = dsc.hg_matrix(dirs, g, "flatland")
        series = 1.0 + 2.0 * sum(g ** k * np.cos(k * dth) for k in range(1, 600))
        assert np.allclose(P, series, rtol=1e-11, atol=1e-11)


def test_sphere_kernel_is_the_legendre_series():
    # (1-g^2)/(1+g^2-2g mu)^{3/2} = sum_l (2l+1) g^l P_l(mu)
    dirs, _ = quadrature.sphere_product(4, 6)
    g = 0.6
    P = dsc.hg_matrix(dirs, g, "sphere")
    mu = np.clip(dirs @ dirs.T, -1, 1)
    coef = np.array([(2 * l + 1) * g ** l for l in range(250)])
    series = np.polynomial.legendre.legval(mu, coef)
    assert np.allclose(P, series, rtol=1e-10)


@pytest.mark.parametrize("quad,g,kind", [(quadrature.circle(16), 0.5, "flatland"),
                                         (quadrature.circle(64), 0.9, "flatland"),
                                         (quadrature.sphere_product(8, 12), 0.8, "sphere"),
                                         (quadrature.s2_xy(), 0.3, "sphere"),
                                         (quadrature.circle(32), -0.4, "flatland")])
def test_scatter_matrix_conserves(quad, g, kind):
    dirs, w = quad
    S, K = dsc.scatter_matrix(dirs, w, g, kind)
    assert np.allclose(S.sum(axis=1), 1.0, atol=1e-14)          # rows
    assert np.allclose(w @ S, w, atol=1e-14)                     # w-weighted columns
    assert np.allclose(K, K.T, atol=1e-13 * np.abs(K).max())
    assert (S > 0).all()


@pytest.mark.parametrize("N,g", [(16, 0.5), (32, 0.9), (8, -0.3)])
def test_flatland_spectrum_on_the_circle(N, g):
    dirs, w = quadrature.circle(N)
    S, _ = dsc.scatter_matrix(dirs, w, g, "flatland")
    lam = np.sort(np.linalg.eigvals(S).real)
    k = np.arange(N)
    expect = np.sort((g ** k + g ** (N - k)) / (1.0 + g ** N))
    assert np.allclose(lam, expect, atol=2e-14)
    # mean scattering cosine is the dipole eigenvalue
    mc = (S * (dirs @ dirs.T)).sum(axis=1)
    assert np.allclose(mc, (g + g ** (N - 1)) / (1 + g ** N), atol=1e-14)


def test_isotropic_scattering_is_the_average():
    dirs, w = quadrature.circle(16)
    S, _ = dsc.scatter_matrix(dirs, w, 0.0)
    assert np.allclose(S, np.tile(w, (16, 1)), atol=1e-15)


# --------------------------------------------------- psi == 1 (pin 1) ---

@pytest.mark.parametrize("kw", [dict(g=0.5, eps=0.01), dict(g=0.9, eps=1e-3),
                                dict(g=0.0, eps=1.0),
                                dict(dim=3, ndir=8, g=0.7, eps=0.05, n=6, kind="sphere")])
def test_unit_inflow_gives_unit_solution(kw):
    kw = dict(kw)
    n = kw.pop("n", 10)
    prob = problems.make(n=n, sigma_a=0.0, q=0.0, inflow="uniform", **kw)
    D = dsc.Discretisation(prob)
    b = dsc.rhs(D)
    L1 = dsc.apply_L(D, np.ones((D.N, D.cells)))
    assert np.max(np.abs(L1 - b)) <= 1e-12 * np.max(np.abs(b))
    if D.n <= 4096:
        psi = direct.lu_solve(D, b)
        assert np.max(np.abs(psi - 1.0)) < 1e-9


# ------------------------------------------- exponential decay (pin 2) ---

@pytest.mark.parametrize("eps", [1.0, 0.5])
def test_absorbing_ray_closed_form(eps):
    rng = np.random.default_rng(11)
    n = 16
    st = rng.uniform(0.5, 3.0, (n, n))
    prob = problems.make(n=n, quad=quadrature.axis4(), sigma_t=st, sigma_a=st / eps ** 2,
                         q=0.0, eps=eps, inflow="left")
    D = dsc.Discretisation(prob)
    assert np.all(D.sS == 0.0)
    x, info = krylov.fgmres(lambda v: dsc.apply_L(D, v).reshape(-1), dsc.rhs(D).reshape(-1),
                            restart=60, rtol=1e-14, max_iters=2000)
    psi = x.reshape(4, n, n)
    h = 1.0 / n
    expect = np.cumprod(1.0 / (1.0 + (st / eps) * h), axis=1)      # along x, per row
    assert np.allclose(psi[0], expect, rtol=1e-12, atol=1e-15)
    assert np.max(np.abs(psi[1:])) < 1e-14


def test_absorbing_ray_first_order_convergence():
    errs = []
    for n in (16, 32, 64, 128):
        prob = problems.make(n=n, quad=quadrature.axis4(), sigma_t=1.0, sigma_a=1.0, q=0.0,
                             eps=1.0, inflow="left")
        D = dsc.Discretisation(prob)
        psi = direct.sweep_solve(D).reshape(4, n, n)[0]
        x = (np.arange(n) + 0.5) / n
        errs.append(np.max(np.abs(psi[0] - np.exp(-x))))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((rates > 0.9) & (rates < 1.1))


# ----------------------------------------------- dense LU (pin 4) ---

def _small(**kw):
    base = dict(n=8, ndir=8, g=0.5, eps=0.1, inflow="random", seed=4)
    base.update(kw)
    return dsc.Discretisation(problems.make(**base))


def test_diagonal_and_sign_structure():
    D = _small()
    A = direct.dense_matrix(D)
    assert np.allclose(np.diag(A), dsc.diagonal(D).reshape(-1), rtol=1e-14)
    off = A - np.diag(np.diag(A))
    assert off.max() <= 0.0                 # upwind + positive scattering: an M-matrix pattern
    assert np.all(np.diag(A) > 0)


def test_fgmres_equals_lu():
    D = _small()
    b = dsc.rhs(D).reshape(-1)
    ref = direct.lu_solve(D).reshape(-1)
    x, info = krylov.fgmres(lambda v: dsc.apply_L(D, v).reshape(-1), b, restart=20, rtol=1e-13,
                            max_iters=5000)
    assert info["converged"]
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-10


def test_exact_preconditioner_converges_in_one_step():
    D = _small()
    A = direct.dense_matrix(D)
    Ainv = np.linalg.inv(A)
    b = dsc.rhs(D).reshape(-1)
    x, info = krylov.fgmres(lambda v: A @ v, b, precond=lambda v: Ainv @ v, restart=10, rtol=1e-12)
    assert info["iterations"] == 1 and info["converged"]


def test_full_krylov_space_terminates():
    D = _small(n=4, ndir=4, eps=0.05)
    b = dsc.rhs(D).reshape(-1)
    x, info = krylov.fgmres(lambda v: dsc.apply_L(D, v).reshape(-1), b, restart=D.n, rtol=1e-10,
                            max_iters=D.n)
    assert info["converged"] and info["iterations"] <= D.n


# ------------------------------------------ sweeps / source iteration (pin 5) ---

def test_sweep_equals_fgmres_without_scattering():
    rng = np.random.default_rng(5)
    st = rng.uniform(0.5, 4.0, (10, 10))
    D = dsc.Discretisation(problems.make(n=10, ndir=12, sigma_t=st, sigma_a=st, eps=1.0,
                                         inflow="random", q=0.3))
    ref = direct.sweep_solve(D)
    x, _ = krylov.fgmres(lambda v: dsc.apply_L(D, v).reshape(-1), dsc.rhs(D).reshape(-1),
                         restart=40, rtol=1e-14, max_iters=4000)
    assert np.linalg.norm(x - ref.reshape(-1)) / np.linalg.norm(ref) < 1e-12


def test_source_iteration_equals_fgmres():
    D = dsc.Discretisation(problems.make(n=10, ndir=8, g=0.5, eps=1.0, sigma_a=0.4,
                                         inflow="random", seed=9))
    ref, its = direct.source_iteration(D, tol=1e-15)
    x, _ = krylov.fgmres(lambda v: dsc.apply_L(D, v).reshape(-1), dsc.rhs(D).reshape(-1),
                         restart=40, rtol=1e-14, max_iters=4000)
    assert np.linalg.norm(x - ref.reshape(-1)) / np.linalg.norm(ref) < 1e-12


# ---------------------------------------------- particle balance (pin 6) ---

@pytest.mark.parametrize("dim", [2, 3])
def test_discrete_particle_balance(dim):
    if dim == 2:
        D = _small(n=8, ndir=8, g=0.7, eps=0.2, q=0.7)
    else:
        D = dsc.Discretisation(problems.make(dim=3, n=4, ndir=8, g=0.6, eps=0.3, q=0.5,
                                             inflow="random", kind="sphere"))
    psi = direct.lu_solve(D).reshape(D.N, D.nz, D.ny, D.nx)
    hd = D.h ** D.dim
    hd1 = D.h ** (D.dim - 1)
    out = 0.0
    inc = 0.0
    for m in range(D.N):
        for a in range(D.dim):
            ua = D.dirs[m, a]
            if ua == 0:
                continue
            ax = 3 - a
            last = [slice(None)] * 4
            last[0] = m
            last[ax] = -1 if ua > 0 else 0
            out += D.w[m] * abs(ua) * hd1 * psi[tuple(last)].sum()
            face = 2 * a + (0 if ua > 0 else 1)
            inc += D.w[m] * abs(ua) * hd1 * dsc.face_values(D, face, m).sum()
    phi = dsc.scalar_flux(D, psi)
    lhs = out + hd * (D.sA * phi).sum()
    rhs_ = hd * D.qh.sum() + inc
    assert abs(lhs - rhs_) <= 1e-12 * abs(rhs_)


# ------------------------------------------------ diffusion limit (pin 7) ---

def test_diffusion_limit_isotropy_and_scalar_flux():
    n, ndir = 10, 8
    isos, errs = [], []
    base = dict(n=n, ndir=ndir, g=0.5, sigma_a=0.5, inflow="left", seed=2)
    D0 = dsc.Discretisation(problems.make(eps=1.0, q=0.0, **base))
    phi0 = direct.isotropic_limit(D0, dsc.rhs(D0))
    for eps in (1e-3, 1e-4, 1e-5):
        D = dsc.Discretisation(problems.make(eps=eps, q=1.0, **base))
        psi = direct.lu_solve(D)
        isos.append(np.linalg.norm(psi - D.S @ psi) / np.linalg.norm(psi))
        errs.append(np.linalg.norm(dsc.scalar_flux(D, psi) - phi0) / np.linalg.norm(phi0))
    for seq in (isos, errs):
        slopes = np.log10(np.array(seq[:-1]) / np.array(seq[1:]))
        assert np.all((slopes > 0.9) & (slopes < 1.1)), seq
    assert errs[-1] < 1e-4


# ------------------------------------------------ mirror symmetry (pin 8) ---

def test_mirror_symmetry():
    rng = np.random.default_rng(8)
    st = rng.uniform(0.5, 2.0, (8, 8))
    st = 0.5 * (st + st[:, ::-1])
    D = dsc.Discretisation(problems.make(n=8, ndir=8, sigma_t=st, g=0.6, eps=0.3,
                                         inflow="uniform", q=1.0))
    psi = direct.lu_solve(D).reshape(D.N, 8, 8)
    mirror = [int(np.argmin(np.linalg.norm(D.dirs - D.dirs[m] * [-1, 1, 1], axis=1)))
              for m in range(D.N)]
    for m in range(D.N):
        assert np.allclose(psi[m], psi[mirror[m]][:, ::-1], rtol=1e-12, atol=1e-14)


# --------------------------------------------- network semantics (pin 9) ---

def test_bilinear_prolongation_reproduces_linear_functions():
    C, n = 3, 8
    k = np.array([1, 3, 3, 1]) / 4.0
    W = np.zeros((C, C, 4, 4))
    for c in range(C):
        W[c, c] = np.outer(k, k)
    Xc = (np.arange(n) + 0.5) * 2.0 / (2 * n)
    coarse = np.stack([1.0 + 2.0 * Xc[None, :] - 0.5 * Xc[:, None] for _ in range(C)])
    fine = network.conv_transpose4(coarse, W)
    xf = (np.arange(2 * n) + 0.5) / (2 * n)
    expect = 1.0 + 2.0 * xf[None, :] - 0.5 * xf[:, None]
    assert np.allclose(fine[:, 1:-1, 1:-1], expect[None, 1:-1, 1:-1], atol=1e-14)


def test_full_weighting_restriction_keeps_constants():
    C = 2
    k = np.array([1, 2, 1]) / 4.0
    W = np.zeros((C, C, 3, 3))
    for c in range(C):
        W[c, c] = np.outer(k, k)
    out = network.conv3(np.full((C, 8, 8), 3.0), W, stride=2)
    assert np.allclose(out[:, 1:, 1:], 3.0, atol=1e-15)


@pytest.mark.parametrize("dim", [2, 3])
def test_vcycle_is_linear(dim):
    prob, blob = problems.net_problem(dim)
    P = osolve.Problem(prob, blob)
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal((2, P.D.n))
    lhs = P.precond(2.0 * u - 3.0 * v)
    rhs_ = 2.0 * P.precond(u) - 3.0 * P.precond(v)
    assert np.linalg.norm(lhs - rhs_) <= 1e-12 * np.linalg.norm(lhs)


def _identity_net_problem():
    # one level, one smoothing step, A = 0, a = 0, a^{-1} = 1, B = centre-tap identity,
    # W_in = W_out = I (c0 = N), s = 1: u = B * (a^{-1} f) = v / d and z = 2 v / d
    prob = problems.make(n=8, ndir=8, g=0.5, eps=0.1,
                         mg=dict(c0=8, levels=1, nu_pre=0, nu_post=0, nu_coarse=1, coef_ch=3, seed=1))
    hdr, t = configs.problem_weights(prob)
    T = weights.tag
    t[T(weights.K_A, 0)][:] = 0
    t[T(weights.K_HAW, 0)][:] = 0
    t[T(weights.K_HAB, 0)][:] = 0
    t[T(weights.K_HIW, 0)][:] = 0
    t[T(weights.K_HIB, 0)][:] = 1
    B = t[T(weights.K_BC, 0, 0)]
    B[:] = 0
    for c in range(8):
        B[c, c, 1, 1] = 1.0
    return osolve.Problem(prob, weights.pack_mgn1(hdr, t))


def test_vcycle_identity_weights_give_twice_jacobi():
    P = _identity_net_problem()
    v = np.random.default_rng(1).standard_normal(P.D.n)
    assert np.allclose(P.precond(v), 2.0 * v / P.diag.reshape(-1), rtol=1e-14)


def test_bf16_vcycle_identity_weights_and_homogeneity():
    # with identity weights only the smoother's input is rounded: z = v/d + bf16(v/d)
    P = _identity_net_problem()
    v = np.random.default_rng(2).standard_normal(P.D.n)
    vt = v / P.diag.reshape(-1)
    assert np.allclose(P.precond_bf16(v), vt + network.round_bf16(vt), rtol=1e-15, atol=0)
    # rounding commutes with scaling by 2, so the rounded V-cycle is exactly homogeneous
    prob, blob = problems.net_problem(2)
    Q = osolve.Problem(prob, blob)
    w = np.random.default_rng(4).standard_normal(Q.D.n)
    z = Q.precond_bf16(w)
    assert np.array_equal(Q.precond_bf16(2.0 * w), 2.0 * z)
    # and it moves the V-cycle by about the bfloat16 unit roundoff, not by zero or by O(1)
    e = np.linalg.norm(z - Q.precond(w)) / np.linalg.norm(Q.precond(w))
    assert 2.0 ** -12 < e < 2.0 ** -4


def test_mgn1_reader_rejects_corrupt_blobs():
    prob, blob = problems.net_problem(2)
    network.Net(blob)
    for bad in (blob[:100], b"XGN1" + blob[4:], blob + b"\0\0\0\0", blob[:-4]):
        with pytest.raises(network.FormatError):
            network.Net(bad)
    hdr, t = configs.problem_weights(prob)
    k = next(iter(t))
    del t[k]
    with pytest.raises(network.FormatError):
        network.Net(weights.pack_mgn1(hdr, t))


# ------------------------------------------------- Arnoldi (pin 10) ---

def test_arnoldi_identities_and_preconditioned_solution():
    prob, blob = problems.net_problem(2)
    P = osolve.Problem(prob, blob)
    rec = []
    x, info = P.solve(rtol=1e-12, restart=15, record=rec)
    assert info["converged"]
    for V, Z, H, j in rec:
        AZ = np.stack([P.apply(z) for z in Z])
        assert np.linalg.norm(AZ.T - V.T @ H) <= 1e-11 * np.linalg.norm(AZ)
        assert np.max(np.abs(V @ V.T - np.eye(V.shape[0]))) < 1e-12
    # preconditioning changes the path, not the answer
    x0, _ = P.solve(rtol=1e-12, restart=15, use_net=False)
    assert np.linalg.norm(x - x0) / np.linalg.norm(x0) < 1e-9


# ------------------------------------ Block-Jacobi comparator (pin 11) ---

@pytest.mark.parametrize("dim", [2, 3])
def test_block_jacobi_blocks_are_the_diagonal_blocks_of_L(dim):
    """The formula-built cell blocks equal the cell-diagonal blocks of the dense
    operator assembled column by column from apply_L."""
    from oracle import comparators
    prob = problems.make(n=3, ndir=8, dim=dim, eps=0.3, seed=5, nz=2 if dim == 3 else None)
    D = dsc.Discretisation(prob)
    A = direct.dense_matrix(D)
    B = comparators.cell_blocks(D)
    for c in range(D.cells):
        idx = np.arange(D.N) * D.cells + c
        assert np.allclose(A[np.ix_(idx, idx)], B[c], rtol=0, atol=1e-12 * np.abs(A).max())


def test_block_jacobi_is_exact_on_one_cell():
    """On a one-cell grid L has no neighbour couplings: Block-Jacobi is L^{-1}."""
    prob = problems.make(n=1, ndir=8, eps=0.05, seed=2, sigma_t=3.0)
    P = osolve.Problem(prob)
    v = np.random.default_rng(3).normal(size=P.D.n)
    z = P.block_jacobi(v)
    exact = np.linalg.solve(direct.dense_matrix(P.D), v)
    assert np.linalg.norm(z - exact) <= 1e-12 * np.linalg.norm(exact)


def test_block_jacobi_without_scattering_is_the_diagonal():
    """sS = 0 (sigma_a = sigma_T / eps^2): each block is diagonal, z = v / (stream + sT)."""
    eps, st = 0.5, 2.0
    prob = problems.make(n=4, ndir=8, eps=eps, sigma_t=st, sigma_a=st / eps ** 2, seed=1)
    P = osolve.Problem(prob)
    assert np.abs(P.D.sS).max() < 1e-12
    v = np.random.default_rng(4).normal(size=(P.D.N, P.D.cells))
    stream = np.abs(P.D.dirs[:, :2]).sum(axis=1) / P.D.h
    z = P.block_jacobi(v).reshape(P.D.N, P.D.cells)
    assert np.allclose(z, v / (stream[:, None] + P.D.sT[None, :]), rtol=1e-13, atol=0)


def test_block_jacobi_fgmres_reaches_the_lu_solution():
    prob = problems.make(n=6, ndir=8, eps=0.1, seed=7)
    P = osolve.Problem(prob)
    x, st = P.solve(rtol=1e-12, restart=20, precond="bj")
    assert st["converged"]
    ref = direct.lu_solve(P.D)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-9

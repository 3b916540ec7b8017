"""Pins of the ATFPS oracle (Sec. 2.3) and its filtered loss (Sec. 3.4).

1. The selection of eq. (def_V_delta) in its second form (exp(-|xi| sT h / 2) > delta) equals
   its first form, the max-norm of each basis function evaluated at the cell centre.
2. With delta = 0 nothing is dropped, every face basis spans its directions, and the
   projected conditions are an invertible transformation of the TFPS rows: the ATFPS solution
   is the TFPS solution (a wrong projection, sign or face breaks this).
3. A solution made only of kept modes (a constant plus slowly decaying exponentials of a
   homogeneous medium) satisfies the compressed conditions exactly, so ATFPS reproduces it
   for delta > 0, and layer reconstruction adds nothing.
4. For delta > 0 in the diffusive regime: the error against full TFPS falls with delta, the
   layer reconstruction of eq. (2DAdaptive_TFPS_layer1/2) reduces it (a sign error there
   increases it), and it stays within the a posteriori bound's form delta ||alpha_delta||_inf
   (Theorem posteriori, its constant unknown: checked with constant 1).
5. The filtered loss vanishes at the cell-centre values of the ATFPS smooth solution when no
   cell keeps more functions than there are directions (D_delta then recovers the kept
   coefficients exactly), and is positive for a perturbed field.
"""
import numpy as np
import pytest
import scipy.linalg

import problems
from oracle import atfps, tfps


def _prob(eps, n=12, ndir=8, inflow="left", seed=2, **kw):
    return problems.make(n=n, ndir=ndir, g=0.5, eps=eps, seed=seed, inflow=inflow, **kw)


def test_selection_rule_two_forms():
    A = atfps.ATFPS(_prob(0.02), 1e-2)
    T = A.T
    for c in (0, 17, 143):
        i, j = c % T.I, c // T.I
        centre = ((i + 0.5) * T.h, (j + 0.5) * T.h)
        vals = np.max(np.abs(T.basis_at(c, centre)), axis=0)
        assert np.array_equal(vals > A.delta, A.keep[c])
    assert 0 < A.n < T.n


@pytest.mark.parametrize("eps", [0.5, 0.02])
def test_zero_delta_is_tfps(eps):
    prob = _prob(eps, inflow="random")
    T = tfps.TFPS(prob)
    ref = T.psi_centres(T.solve())
    A = atfps.ATFPS(prob, 0.0)
    assert A.n == T.n
    psi = A.psi_centres(A.reconstruct(A.solve()))
    assert np.max(np.abs(psi - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_kept_mode_solutions_are_exact():
    prob = problems.make(n=8, ndir=8, g=0.4, eps=0.05, sigma_t=2.0, sigma_a=0.4, q=1.0, seed=0,
                         inflow="uniform")
    A0 = atfps.ATFPS(prob, 1e-2)
    D = A0.T.D
    sT, sS, qh = D.sT[0], D.sS[0], D.qh[0]
    B = (sS / sT) * D.S - np.eye(D.N)
    wx, Vx = scipy.linalg.eig(B, np.diag(D.dirs[:, 0]))
    wx, Vx = wx.real, Vx.real
    h = A0.T.h
    kept_x = np.exp(-0.5 * np.abs(wx) * sT * h) > A0.delta
    slow = [k for k in np.argsort(np.abs(wx)) if kept_x[k]][:2]   # two slow x modes, both kept
    assert len(slow) == 2

    def psi_ex(x, y):
        return qh / (sT - sS) + 0.3 * Vx[:, slow[0]] * np.exp(sT * wx[slow[0]] * (x - 0.5)) \
            + 0.2 * Vx[:, slow[1]] * np.exp(sT * wx[slow[1]] * (x - 0.5))

    I = A0.I
    inflow = np.zeros((4, D.N, prob["inflow"].shape[2]))
    for j in range(I):
        yc = (j + 0.5) * h
        inflow[0, :, j], inflow[1, :, j] = psi_ex(0.0, yc), psi_ex(1.0, yc)
        inflow[2, :, j], inflow[3, :, j] = psi_ex(yc, 0.0), psi_ex(yc, 1.0)
    prob = dict(prob, inflow=inflow)
    A = atfps.ATFPS(prob, 1e-2)
    al = A.solve()
    smooth = A.psi_centres(A.scatter(al))
    full = A.psi_centres(A.reconstruct(al))
    ref = np.stack([psi_ex((c % I + 0.5) * h, (c // I + 0.5) * h) for c in range(I * I)], axis=1)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(smooth - ref)) <= 1e-9 * scale
    assert np.max(np.abs(full - ref)) <= 1e-9 * scale


@pytest.mark.slow
def test_error_falls_with_delta_and_reconstruction_helps():
    prob = _prob(0.02)
    T = tfps.TFPS(prob)
    ref = T.psi_centres(T.solve())
    scale = np.max(np.abs(ref))
    errs = []
    for delta in (1e-1, 1e-2, 1e-3, 1e-4):
        A = atfps.ATFPS(prob, delta)
        al = A.solve()
        e_full = np.max(np.abs(A.psi_centres(A.reconstruct(al)) - ref))
        e_smooth = np.max(np.abs(A.psi_centres(A.scatter(al)) - ref))
        assert e_full < e_smooth
        assert e_full <= delta * np.max(np.abs(al))
        errs.append(e_full / scale)
    assert all(a > b for a, b in zip(errs, errs[1:]))


def test_filtered_loss_vanishes_at_the_smooth_solution():
    prob = _prob(0.005)
    A = atfps.ATFPS(prob, 1e-2)
    assert max(len(k) for k in A.kidx) <= A.N
    Am, b = A.assemble()
    al = A.solve()
    psi = A.psi_centres(A.scatter(al))
    bn = np.linalg.norm(b)
    assert A.filtered_loss(psi, Am, b) <= 1e-10 * bn
    pert = psi + 1e-3 * np.random.default_rng(0).standard_normal(psi.shape)
    assert A.filtered_loss(pert, Am, b) > 1e-6 * bn

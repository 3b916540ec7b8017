"""The PyTorch network used for offline training computes what the library and
the oracle compute: the operator L and the V-cycle with CoeffNet fields, in
FP64 on the CPU, against the oracle on a small problem."""
import numpy as np
import pytest

import problems
from oracle import discretisation as dsc
from oracle import network
from oracle import solve as osolve
from rte_inputs import configs, weights

torch = pytest.importorskip("torch")


def _setup():
    from paper_2604_23265_amd import train_mgnet as T
    prob = problems.make(n=16, ndir=8, eps=0.05, g=0.5, seed=3,
                         mg=dict(c0=16, levels=3, nu_pre=2, nu_post=1, nu_coarse=2, coef_ch=3, seed=11))
    hdr, t = configs.problem_weights(prob)
    blob = weights.pack_mgn1(hdr, t)
    P = osolve.Problem(prob, blob)
    md = T.Medium([prob], P.D.S[None], "cpu", torch.float64)
    net = T.MgNet(hdr, t, "cpu", torch.float64)
    return T, prob, P, md, net


def test_training_operator_is_the_discrete_operator():
    T, prob, P, md, net = _setup()
    psi = np.random.default_rng(1).standard_normal((P.D.N, P.D.cells))
    ref = dsc.apply_L(P.D, psi).reshape(P.D.N, -1)
    got = T.apply_L(torch.as_tensor(psi.reshape(1, P.D.N, P.D.ny, P.D.nx)), md).numpy().reshape(P.D.N, -1)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_training_network_is_the_vcycle():
    T, prob, P, md, net = _setup()
    with torch.no_grad():
        fields = net.coeffnet(md.X)
        a_ref, ai_ref = network.coeffnet(P.net, P.D)
        for l in range(P.net.L):
            assert np.allclose(fields[0][l][0].numpy(), a_ref[l], rtol=1e-12, atol=1e-13)
            assert np.allclose(fields[1][l][0].numpy(), ai_ref[l], rtol=1e-12, atol=1e-13)
        v = np.random.default_rng(2).standard_normal(P.D.n)
        z = net(torch.as_tensor(v.reshape(1, P.D.N, P.D.ny, P.D.nx)), md, fields).numpy().reshape(-1)
    ref = P.precond(v)
    assert np.linalg.norm(z - ref) <= 1e-11 * np.linalg.norm(ref)
    # the blob written back is the blob read
    assert net.blob() == weights.pack_mgn1(*configs.problem_weights(prob))


def test_best_keeper_restores_the_best_window_after_divergence():
    from paper_2604_23265_amd import train_mgnet as T
    w = torch.zeros(3)
    keeper = T.BestKeeper(window=4, slack=1.5)
    hist = []
    for it in range(16):
        w += 1.0                                          # the parameters move every step
        hist.append(1.0 / (it + 1) if it < 8 else 1e30)   # loss falls, then blows up
        keeper.update(it, hist, [w])
    step, loss = keeper.finish(hist, [w])
    assert step == 7 and abs(loss - np.mean([1 / 5, 1 / 6, 1 / 7, 1 / 8])) < 1e-12
    assert torch.equal(w, torch.full((3,), 8.0))        # the parameters of step 7
    # a run that ends at its best keeps its final parameters
    w2 = torch.zeros(2)
    k2, h2 = T.BestKeeper(window=4), []
    for it in range(8):
        w2 += 1.0
        h2.append(1.0 / (it + 1))
        k2.update(it, h2, [w2])
    assert k2.finish(h2, [w2])[0] == 7 and torch.equal(w2, torch.full((2,), 8.0))

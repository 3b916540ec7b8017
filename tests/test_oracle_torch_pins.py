"""Pins of the FP64 oracle's convolutions and CoeffNet against PyTorch's routines.

PyTorch's CPU convolutions (float64) and its bfloat16 conversion are an
independent route to the same values; the module is skipped without torch.
"""
import numpy as np
import pytest

import problems
from oracle import network
from oracle import discretisation as dsc

torch = pytest.importorskip("torch")
F = torch.nn.functional


@pytest.mark.parametrize("dim,stride", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_conv3_is_pytorch_cross_correlation(dim, stride):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5,) + (8,) * dim)
    W = rng.standard_normal((7, 5) + (3,) * dim)
    fn = F.conv2d if dim == 2 else F.conv3d
    ref = fn(torch.from_numpy(x)[None], torch.from_numpy(W), stride=stride, padding=1)[0].numpy()
    assert np.allclose(network.conv3(x, W, stride), ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_conv_transpose4_is_pytorch(dim):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((6,) + (4,) * dim)
    W = rng.standard_normal((6, 3) + (4,) * dim)
    fn = F.conv_transpose2d if dim == 2 else F.conv_transpose3d
    ref = fn(torch.from_numpy(x)[None], torch.from_numpy(W), stride=2, padding=1)[0].numpy()
    out = network.conv_transpose4(x, W)
    assert out.shape == ref.shape
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_coeffnet_is_the_pytorch_pyramid(dim):
    prob, blob = problems.net_problem(dim)
    D = dsc.Discretisation(prob)
    net = network.Net(blob)
    a, ainv = network.coeffnet(net, D)
    conv = F.conv2d if dim == 2 else F.conv3d
    sh = network.spatial_shape(D)
    X = torch.from_numpy(np.stack([np.log(D.sT), D.sA / D.sT, np.log(D.eps)]).reshape((3,) + sh))[None]
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    Fm = X
    for l in range(net.L):
        Fm = torch.relu(conv(Fm, T(net.CW[l]), T(net.CB[l]), stride=1 if l == 0 else 2, padding=1))
        wa = T(net.HAW[l]).reshape(net.HAW[l].shape + (1,) * dim)
        wi = T(net.HIW[l]).reshape(net.HIW[l].shape + (1,) * dim)
        assert np.allclose(a[l], conv(Fm, wa, T(net.HAB[l]))[0].numpy(), rtol=1e-12, atol=1e-12)
        assert np.allclose(ainv[l], conv(Fm, wi, T(net.HIB[l]))[0].numpy(), rtol=1e-12, atol=1e-12)


def test_round_bf16_matches_torch_bfloat16():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(200000) * np.exp(rng.uniform(-30, 30, 200000))
    # bfloat16 spacing near 1 is 2^-7: 1 + 2^-8 and 1 + 3 2^-8 are ties, rounded to even
    x[:4] = [0.0, -2.5, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8]
    r = network.round_bf16(x)
    t = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(r, t)
    assert r[2] == 1.0 and r[3] == 1.0 + 2.0 ** -6 and r[1] == -2.5

"""Seeded input generators: determinism and the properties callers rely on."""
import hashlib

import numpy as np
import pytest

from rte_inputs import configs, media, quadrature, weights


def _digest(prob):
    h = hashlib.sha256()
    for k in ("dirs", "weights", "sigma_t", "sigma_a", "q"):
        h.update(np.ascontiguousarray(prob[k]).tobytes())
    if prob["inflow"] is not None:
        h.update(prob["inflow"].tobytes())
    h.update(np.atleast_1d(prob["eps"]).tobytes())
    return h.hexdigest()


@pytest.mark.parametrize("make", [lambda: configs.c1(), lambda: configs.c2(0, n=64, ndir=16),
                                  lambda: configs.c3_request(5), lambda: configs.p0(1),
                                  lambda: configs.c5(0, n=8, n_mu=2, n_phi=4)])
def test_same_seed_same_arrays(make):
    assert _digest(make()) == _digest(make())


def test_different_seeds_differ():
    assert _digest(configs.c2(0, n=32, ndir=8)) != _digest(configs.c2(1, n=32, ndir=8))


@pytest.mark.parametrize("quad,second", [(quadrature.circle(16), 0.5), (quadrature.circle(64), 0.5),
                                         (quadrature.sphere_product(8, 12), 1.0 / 3.0),
                                         (quadrature.s2_xy(), None), (quadrature.axis4(), 0.5)])
def test_quadrature_moments(quad, second):
    dirs, w = quad
    assert np.allclose(np.linalg.norm(dirs, axis=1), 1.0, atol=1e-15)
    assert abs(w.sum() - 1.0) < 1e-14
    assert np.allclose(w @ dirs[:, :2], 0.0, atol=1e-15)     # x-y sets keep the z > 0 half
    if second is not None:
        assert abs(w @ dirs[:, 0] ** 2 - second) < 1e-14


def test_sphere_set_integrates_polynomials():
    dirs, w = quadrature.sphere_product(8, 12)
    # Gauss-Legendre with 8 nodes integrates mu^k exactly for k <= 15: mean of mu^4 is 1/5.
    assert abs(w @ dirs[:, 2] ** 4 - 0.2) < 1e-14
    assert dirs.shape == (96, 3)


def test_grf_normalisation_and_correlation():
    rng = np.random.default_rng(3)
    f = media.gaussian_random_field((128, 128), 0.5, 0.1, rng)
    assert abs(f.mean()) < 1e-12 and abs(f.std() - 0.5) < 1e-12
    # correlation at lag 0.1 (13 cells) should be near exp(-1/2), far below at lag 0.4
    c = lambda lag: np.mean(f[:, :-lag] * f[:, lag:]) / f.var()
    assert 0.35 < c(13) < 0.85 and abs(c(51)) < 0.3


def test_checkerboard_layout():
    st, black = media.checkerboard(512, 8, 100.0, 1.0)
    assert st[0, 0] == 100.0 and st[0, 64] == 1.0 and st[64, 64] == 100.0
    assert black.mean() == 0.5


def test_c1_inclusion_is_cell_aligned():
    p = configs.c1()
    st = p["sigma_t"].reshape(32, 32)
    assert st[12, 12] == 10 and st[19, 19] == 10 and st[11, 12] == 1 and st[20, 20] == 1
    assert (st == 10).sum() == 64


def test_polynomial_medium_gap():
    rng = np.random.default_rng(0)
    for _ in range(5):
        st, sa = media.polynomial_medium(32, rng)
        assert (st - sa).min() >= 0.2 - 1e-12


def test_mgn1_layout_and_order():
    hdr, t = weights.seeded_weights(2, 8, 8, 2, seed=1)
    blob = weights.pack_mgn1(hdr, t)
    assert blob[:4] == b"MGN1"
    # header + every record is tag, rank, dims, float32 payload
    size = 48 + sum(8 + 4 * a.ndim + 4 * a.size for a in t.values())
    assert len(blob) == size
    assert np.allclose(t[weights.tag(weights.K_WIN)], np.eye(8))


def test_trained_weights_record():
    """The committed trained weights are the ones their record describes and
    parse as an MGN1 network of the C2 shape."""
    import hashlib
    import json
    import os
    from oracle import network
    root = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2604_23265_amd", "weights")
    blob = open(os.path.join(root, "c2_mgnet.mgn1"), "rb").read()
    rec = json.load(open(os.path.join(root, "c2_mgnet.json")))
    assert hashlib.sha256(blob).hexdigest() == rec["sha256"]
    net = network.Net(blob)
    hdr, _ = configs.problem_weights(configs.c2(0))
    for k in ("dim", "ndir", "c0", "levels", "nu_pre", "nu_post", "nu_coarse", "coef_ch"):
        assert net.hdr[k] == hdr[k]


@pytest.mark.parametrize("N", [16, 32])
def test_serving_weights_records(N):
    import hashlib
    import json
    import os
    from oracle import network
    root = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2604_23265_amd", "weights")
    blob = open(os.path.join(root, "c3_n%d.mgn1" % N), "rb").read()
    rec = json.load(open(os.path.join(root, "c3_n%d.json" % N)))
    assert hashlib.sha256(blob).hexdigest() == rec["sha256"]
    net = network.Net(blob)
    p = configs.c3_request(0, ndir_choices=(N,))
    hdr, _ = configs.problem_weights(p)
    for k in ("dim", "ndir", "c0", "levels", "nu_pre", "nu_post", "nu_coarse", "coef_ch"):
        assert net.hdr[k] == hdr[k]

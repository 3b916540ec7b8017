"""Small problem builders shared by the tests (inputs only; no solver arithmetic)."""
import numpy as np

from rte_inputs import configs, media, quadrature


def make(n=16, ndir=8, dim=2, g=0.5, eps=0.1, sigma_t=None, sigma_a=0.05, q=1.0,
         inflow="left", kind="auto", quad=None, seed=0, mg=None, nz=None):
    """A small problem dict on an n^dim grid with a seeded lognormal sigma_T by default."""
    rng = np.random.default_rng(seed)
    if quad is None:
        dirs, w = quadrature.circle(ndir) if dim == 2 else quadrature.sphere_product(2, ndir // 2)
    else:
        dirs, w = quad
    shape = (n, n) if dim == 2 else (nz or n, n, n)
    cells = int(np.prod(shape))
    if sigma_t is None:
        st = media.lognormal_field(shape, 0.5, 0.2, rng)
    elif np.isscalar(sigma_t):
        st = np.full(shape, float(sigma_t))
    else:
        st = np.asarray(sigma_t, float)
    sa = np.full(shape, float(sigma_a)) if np.isscalar(sigma_a) else np.asarray(sigma_a, float)
    qq = np.full(shape, float(q)) if np.isscalar(q) else np.asarray(q, float)
    nn = (n, n, 1) if dim == 2 else (n, n, nz or n)
    if inflow == "left":
        inf = configs.left_unit_inflow(nn, dim, dirs)
    elif inflow == "uniform":
        inf = configs.uniform_inflow(nn, dim, dirs)
    elif inflow == "random":
        fc = max(configs.face_cells(nn, dim, f) for f in range(2 * dim))
        inf = rng.uniform(0.5, 1.5, (2 * dim, dirs.shape[0], fc))
    else:
        inf = None
    if mg is None:
        mg = dict(c0=dirs.shape[0], levels=2, nu_pre=2, nu_post=2, nu_coarse=2, coef_ch=3, seed=seed + 77)
    assert st.size == cells
    return configs._problem("test", dim, nn, dirs, w, g, kind, st, sa, qq, eps, inf, mg,
                            dict(restart=30, rtol=1e-10, max_iters=20000))


def blob_for(prob):
    from rte_inputs import weights
    hdr, t = configs.problem_weights(prob)
    return weights.pack_mgn1(hdr, t)


def net_problem(dim=2):
    """A small problem with a 3-level (2D) or 2-level (3D) seeded MgNet, and its MGN1 blob."""
    if dim == 2:
        prob = make(n=16, ndir=8, g=0.5, eps=0.05, seed=3,
                    mg=dict(c0=8, levels=3, nu_pre=2, nu_post=2, nu_coarse=2, coef_ch=3, seed=12))
    else:
        prob = make(dim=3, n=8, ndir=8, g=0.5, eps=0.05, seed=3, kind="sphere",
                    mg=dict(c0=4, levels=2, nu_pre=1, nu_post=2, nu_coarse=1, coef_ch=3, seed=13))
    return prob, blob_for(prob)

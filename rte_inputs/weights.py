"""Seeded MgNet/CoeffNet weights and the MGN1 container that carries them.

MGN1 is a little-endian binary blob:

  header  : char[4] "MGN1"; uint32 version (=1); uint32 dim, ndir, c0, levels,
            nu_pre, nu_post, nu_coarse, coef_ch, flags, n_tensors
  tensors : n_tensors records of
            uint32 tag; uint32 rank; uint32 dims[rank]; float32 data[prod(dims)]

tag = (kind << 16) | (level << 8) | index.  Kinds and shapes (K = (3,)*dim,
K4 = (4,)*dim, C_l = c0 * 2^l, c_l = coef_ch * 2^l, L = levels):

   1 W_in      [c0, ndir]                       1x1 lift
   2 W_out     [ndir, c0]                       1x1 projection
   3 s         [1]                              skip scale
   4 A_l       [C_l, C_l, *K]                   operator conv, all levels
   5 Bpre_l,i  [C_l, C_l, *K]   l < L-1, i < nu_pre
   6 Bpost_l,i [C_l, C_l, *K]   l < L-1, i < nu_post
   7 Bc_i      [C_l, C_l, *K]   l = L-1, i < nu_coarse
   8 R_l       [C_l+1, C_l, *K] l < L-1           stride-2 restriction
   9 Pr_l      [C_l+1, C_l, *K4] l < L-1          stride-2 transposed conv
  10 CW_l      [c_l, 3 or c_l-1, *K]              CoeffNet conv (stride 2 for l >= 1)
  11 CB_l      [c_l]                              its bias
  12 HAW_l     [C_l, c_l]    13 HAB_l [C_l]       head for a^[l]
  14 HIW_l     [C_l, c_l]    15 HIB_l [C_l]       head for a^{-1,[l]}

Weight layouts follow the PyTorch conventions (conv: [out, in, k...],
transposed conv: [in, out, k...]).  This module draws random numbers and
serialises them; it evaluates no network.
"""
import struct

import numpy as np

MAGIC = b"MGN1"
VERSION = 1

K_WIN, K_WOUT, K_S, K_A, K_BPRE, K_BPOST, K_BC, K_R, K_PR = 1, 2, 3, 4, 5, 6, 7, 8, 9
K_CW, K_CB, K_HAW, K_HAB, K_HIW, K_HIB = 10, 11, 12, 13, 14, 15


def tag(kind, level=0, index=0):
    return (kind << 16) | (level << 8) | index


def seeded_weights(dim, ndir, c0, levels, nu_pre=2, nu_post=2, nu_coarse=2,
                   coef_ch=3, seed=0):
    """Draw a full weight set from PCG64(seed).

    Lift/projection: identity when c0 == ndir, else orthonormal rows from a QR
    factorisation, with W_out = W_in^T.  A ~ N(0, 1/fan_in); B, R, Pr ~
    N(0, 0.01/fan_in); s = 1.  CoeffNet convs Kaiming-normal with small
    biases; heads small, the a^{-1} head biased towards 1.
    """
    rng = np.random.default_rng(seed)
    k3 = (3,) * dim
    k4 = (4,) * dim
    taps3 = 3 ** dim
    hdr = dict(dim=dim, ndir=ndir, c0=c0, levels=levels, nu_pre=nu_pre,
               nu_post=nu_post, nu_coarse=nu_coarse, coef_ch=coef_ch, flags=0)
    t = {}
    if c0 == ndir:
        win = np.eye(c0)
    else:
        g = rng.standard_normal((max(c0, ndir), min(c0, ndir)))
        q, _ = np.linalg.qr(g)
        win = q if c0 > ndir else q.T          # [c0, ndir]
    t[tag(K_WIN)] = win
    t[tag(K_WOUT)] = win.T.copy()
    t[tag(K_S)] = np.ones(1)
    for l in range(levels):
        C = c0 << l
        t[tag(K_A, l)] = rng.normal(0, np.sqrt(1.0 / (C * taps3)), (C, C) + k3)
        if l < levels - 1:
            for i in range(nu_pre):
                t[tag(K_BPRE, l, i)] = rng.normal(0, np.sqrt(0.01 / (C * taps3)), (C, C) + k3)
            for i in range(nu_post):
                t[tag(K_BPOST, l, i)] = rng.normal(0, np.sqrt(0.01 / (C * taps3)), (C, C) + k3)
            t[tag(K_R, l)] = rng.normal(0, np.sqrt(0.01 / (C * taps3)), (2 * C, C) + k3)
            t[tag(K_PR, l)] = rng.normal(0, np.sqrt(0.01 / (2 * C * 2 ** dim)), (2 * C, C) + k4)
        else:
            for i in range(nu_coarse):
                t[tag(K_BC, l, i)] = rng.normal(0, np.sqrt(0.01 / (C * taps3)), (C, C) + k3)
    for l in range(levels):
        c = coef_ch << l
        cin = 3 if l == 0 else (coef_ch << (l - 1))
        C = c0 << l
        t[tag(K_CW, l)] = rng.normal(0, np.sqrt(2.0 / (cin * taps3)), (c, cin) + k3)
        t[tag(K_CB, l)] = rng.normal(0, 0.01, (c,))
        t[tag(K_HAW, l)] = rng.normal(0, np.sqrt(0.01 / c), (C, c))
        t[tag(K_HAB, l)] = rng.normal(0, 0.1, (C,))
        t[tag(K_HIW, l)] = rng.normal(0, np.sqrt(0.01 / c), (C, c))
        t[tag(K_HIB, l)] = 1.0 + rng.normal(0, 0.1, (C,))
    return hdr, {k: np.asarray(v, dtype=np.float32) for k, v in t.items()}


def pack_mgn1(hdr, tensors, order=None):
    """Serialise a header dict and {tag: float32 array} into an MGN1 blob."""
    keys = list(tensors.keys()) if order is None else list(order)
    out = [MAGIC, struct.pack("<I", VERSION)]
    out.append(struct.pack("<10I", hdr["dim"], hdr["ndir"], hdr["c0"], hdr["levels"],
                           hdr["nu_pre"], hdr["nu_post"], hdr["nu_coarse"],
                           hdr["coef_ch"], hdr.get("flags", 0), len(keys)))
    for k in keys:
        a = np.ascontiguousarray(tensors[k], dtype="<f4")
        out.append(struct.pack("<II", k, a.ndim))
        out.append(struct.pack("<%dI" % a.ndim, *a.shape))
        out.append(a.tobytes())
    return b"".join(out)

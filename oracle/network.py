"""CoeffNet and the MgNet V-cycle in FP64 (oracle; test infrastructure).

Architecture (Sec. 3.1-3.3): CoeffNet maps the per-cell medium to, at every
level l, a^[l] (operator information) and a^{-1,[l]} (solution-operator
information), each of shape [C_l, grid / 2^l] with C_l = 2^l C (Sec. 3.2).
MgNet is a V-cycle whose smoother, restriction (stride-2 conv, kernel 3) and
prolongation (stride-2 transposed conv, kernel 4) are convolutions with
angles as channels (Sec. 3.3).  The paper leaves the smoother's exact form,
the head shapes and the lift into C_0 channels open; this file follows one
reading, applied identically at every level:

  input scaling      v~ = v / diag(L)                 (per direction and cell)
  lift               f_0 = W_in v~                    (1x1, N -> C_0)
  smoothing step     r = f - (A * u + a (.) u);  u <- u + B * (a^{-1} (.) r)
  down (l < L-1)     nu_pre steps from u = 0, r_l, f_{l+1} = R_l *_{s2} r_l
  coarsest           nu_coarse steps from u = 0
  up (l = L-2 .. 0)  u_l <- u_l + Pr_l *^T u_{l+1}, then nu_post steps
  output             z = s v~ + W_out u_0

'*' is cross-correlation with zero padding 1 (kernel 3, stride 1 or 2);
'*^T' is the transposed convolution with kernel 4, stride 2, padding 1;
(.) is the elementwise product.  CoeffNet input is
X = [log sT, sA / sT, log eps] (sA = eps sigma_a); F_0 = ReLU(conv3(X) + b),
F_l = ReLU(conv3_s2(F_{l-1}) + b) with coef_ch 2^l channels; the heads are
1x1 convolutions with bias.  MgNet has no bias and no activation, so the
preconditioner is linear in v for a fixed medium.

Spatial arrays are [C, ny, nx] in 2D and [C, nz, ny, nx] in 3D.
"""
import itertools
import struct

import numpy as np

_MAGIC = b"MGN1"


class FormatError(ValueError):
    pass


# ----------------------------------------------------------------- reader ---

def read_mgn1(blob):
    """Parse an MGN1 blob into (header dict, {(kind, level, index): float64 array})."""
    blob = bytes(blob)
    if len(blob) < 48 or blob[:4] != _MAGIC:
        raise FormatError("not an MGN1 blob")
    version, = struct.unpack_from("<I", blob, 4)
    if version != 1:
        raise FormatError("unsupported version")
    vals = struct.unpack_from("<10I", blob, 8)
    names = ("dim", "ndir", "c0", "levels", "nu_pre", "nu_post", "nu_coarse",
             "coef_ch", "flags", "n_tensors")
    hdr = dict(zip(names, vals))
    off = 48
    tensors = {}
    for _ in range(hdr["n_tensors"]):
        if off + 8 > len(blob):
            raise FormatError("truncated tensor record")
        t, rank = struct.unpack_from("<II", blob, off)
        off += 8
        if rank > 8 or off + 4 * rank > len(blob):
            raise FormatError("bad rank")
        dims = struct.unpack_from("<%dI" % rank, blob, off)
        off += 4 * rank
        cnt = int(np.prod(dims)) if rank else 1
        if off + 4 * cnt > len(blob):
            raise FormatError("truncated tensor data")
        a = np.frombuffer(blob, dtype="<f4", count=cnt, offset=off).astype(np.float64)
        off += 4 * cnt
        key = (t >> 16, (t >> 8) & 0xFF, t & 0xFF)
        if key in tensors:
            raise FormatError("duplicate tensor")
        tensors[key] = a.reshape(dims)
    if off != len(blob):
        raise FormatError("trailing bytes")
    return hdr, tensors


class Net:
    """Weights of one MgNet + CoeffNet, addressed by role."""

    def __init__(self, blob):
        hdr, t = read_mgn1(blob)
        self.hdr = hdr
        d = hdr["dim"]
        L = hdr["levels"]
        c0, N, cc = hdr["c0"], hdr["ndir"], hdr["coef_ch"]
        self.dim, self.L, self.N, self.c0, self.cc = d, L, N, c0, cc
        self.nu_pre, self.nu_post, self.nu_coarse = hdr["nu_pre"], hdr["nu_post"], hdr["nu_coarse"]
        k3 = (3,) * d
        k4 = (4,) * d

        def get(kind, shape, level=0, index=0):
            key = (kind, level, index)
            if key not in t:
                raise FormatError("missing tensor %r" % (key,))
            a = t[key]
            if tuple(a.shape) != tuple(shape):
                raise FormatError("tensor %r has shape %r, expected %r" % (key, a.shape, shape))
            return a

        self.W_in = get(1, (c0, N))
        self.W_out = get(2, (N, c0))
        self.s = float(get(3, (1,))[0])
        self.A, self.Bpre, self.Bpost, self.R, self.Pr = [], [], [], [], []
        for l in range(L):
            C = c0 << l
            self.A.append(get(4, (C, C) + k3, l))
            if l < L - 1:
                self.Bpre.append([get(5, (C, C) + k3, l, i) for i in range(self.nu_pre)])
                self.Bpost.append([get(6, (C, C) + k3, l, i) for i in range(self.nu_post)])
                self.R.append(get(8, (2 * C, C) + k3, l))
                self.Pr.append(get(9, (2 * C, C) + k4, l))
        self.Bc = [get(7, ((c0 << (L - 1)),) * 2 + k3, L - 1, i) for i in range(self.nu_coarse)]
        self.CW, self.CB, self.HAW, self.HAB, self.HIW, self.HIB = [], [], [], [], [], []
        for l in range(L):
            c = cc << l
            cin = 3 if l == 0 else cc << (l - 1)
            C = c0 << l
            self.CW.append(get(10, (c, cin) + k3, l))
            self.CB.append(get(11, (c,), l))
            self.HAW.append(get(12, (C, c), l))
            self.HAB.append(get(13, (C,), l))
            self.HIW.append(get(14, (C, c), l))
            self.HIB.append(get(15, (C,), l))
        if len(t) != sum(1 for _ in self._expected_keys()):
            raise FormatError("unexpected extra tensors")

    def _expected_keys(self):
        L = self.L
        yield from [(1, 0, 0), (2, 0, 0), (3, 0, 0)]
        for l in range(L):
            yield (4, l, 0)
            if l < L - 1:
                for i in range(self.nu_pre):
                    yield (5, l, i)
                for i in range(self.nu_post):
                    yield (6, l, i)
                yield (8, l, 0)
                yield (9, l, 0)
        for i in range(self.nu_coarse):
            yield (7, L - 1, i)
        for l in range(L):
            for k in range(10, 16):
                yield (k, l, 0)


# ------------------------------------------------------ convolutions ---

def conv3(x, W, stride=1):
    """Cross-correlation of x [Cin, *S] with W [Cout, Cin, 3, ...], zero padding 1.

    Written out as a sum over taps: out += W[:, :, tap] @ x(shifted by tap).
    """
    d = x.ndim - 1
    xp = np.pad(x, [(0, 0)] + [(1, 1)] * d)
    out_shape = [(s + 2 - 3) // stride + 1 for s in x.shape[1:]]
    out = np.zeros([W.shape[0]] + out_shape)
    for tap in itertools.product(range(3), repeat=d):
        sl = tuple(slice(t, t + stride * (o - 1) + 1, stride) for t, o in zip(tap, out_shape))
        patch = xp[(slice(None),) + sl]
        out += np.tensordot(W[(slice(None), slice(None)) + tap], patch, axes=(1, 0))
    return out


def conv_transpose4(x, W):
    """Transposed convolution, kernel 4, stride 2, padding 1: x [Cin, *S], W [Cin, Cout, 4, ...].

    Input cell i with tap k lands on output index o = 2 i - 1 + k; outputs
    outside [0, 2S) are dropped.  Output shape [Cout, *(2S)].
    """
    d = x.ndim - 1
    S = x.shape[1:]
    full = np.zeros([W.shape[1]] + [2 * s + 2 for s in S])
    for tap in itertools.product(range(4), repeat=d):
        contrib = np.tensordot(W[(slice(None), slice(None)) + tap], x, axes=(0, 0))
        sl = tuple(slice(t, t + 2 * (s - 1) + 1, 2) for t, s in zip(tap, S))
        full[(slice(None),) + sl] += contrib
    return full[(slice(None),) + tuple(slice(1, 2 * s + 1) for s in S)]


def conv1(x, W):
    """1x1 convolution: W [Cout, Cin] applied at every cell."""
    return np.tensordot(W, x, axes=(1, 0))


def _bias(b, d):
    return b.reshape((-1,) + (1,) * d)


# ---------------------------------------------------------- networks ---

def spatial_shape(D):
    return (D.ny, D.nx) if D.dim == 2 else (D.nz, D.ny, D.nx)


def coeffnet(net, D):
    """Per-level (a^[l], a^{-1,[l]}) arrays for the medium of a Discretisation."""
    sh = spatial_shape(D)
    X = np.stack([np.log(D.sT).reshape(sh), (D.sA / D.sT).reshape(sh),
                  np.log(D.eps).reshape(sh)])
    d = D.dim
    a, ainv = [], []
    F = None
    for l in range(net.L):
        if l == 0:
            F = np.maximum(conv3(X, net.CW[0]) + _bias(net.CB[0], d), 0.0)
        else:
            F = np.maximum(conv3(F, net.CW[l], stride=2) + _bias(net.CB[l], d), 0.0)
        a.append(conv1(F, net.HAW[l]) + _bias(net.HAB[l], d))
        ainv.append(conv1(F, net.HIW[l]) + _bias(net.HIB[l], d))
    return a, ainv


def round_bf16(x):
    """x rounded to the nearest bfloat16 value (ties to even), returned as float64.

    bfloat16 keeps the float32 exponent and the top 7 fraction bits; the value
    is first rounded to float32, then the low 16 bits of its encoding are
    rounded away (finite values only).
    """
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def vcycle(net, fields, diag, v, D, bf16=False):
    """z = M(v) for v of shape [N, cells]; `diag` is the diagonal of L, same shape.

    bf16=True rounds the input and the weights of every 3x3 / transposed
    convolution of the V-cycle to bfloat16 (the precision the method runs the
    network in, with wider accumulation), everything else staying FP64: the
    reference for how far rounding alone moves a BF16 V-cycle from the FP64 one.
    """
    a, ainv = fields
    cv3, cvt4 = conv3, conv_transpose4
    if bf16:
        def cv3(x, W, stride=1):
            return conv3(round_bf16(x), round_bf16(W), stride)

        def cvt4(x, W):
            return conv_transpose4(round_bf16(x), round_bf16(W))
    sh = spatial_shape(D)
    L = net.L
    vt = (np.asarray(v).reshape(D.N, D.cells) / diag).reshape((D.N,) + sh)
    f = [None] * L
    u = [None] * L
    f[0] = conv1(vt, net.W_in)

    def residual(l):
        return f[l] - cv3(u[l], net.A[l]) - a[l] * u[l]

    def smooth(l, B):
        r = residual(l)
        u[l] = u[l] + cv3(ainv[l] * r, B)

    for l in range(L - 1):
        u[l] = np.zeros_like(f[l])
        for B in net.Bpre[l]:
            smooth(l, B)
        f[l + 1] = cv3(residual(l), net.R[l], stride=2)
    u[L - 1] = np.zeros_like(f[L - 1])
    for B in net.Bc:
        smooth(L - 1, B)
    for l in range(L - 2, -1, -1):
        u[l] = u[l] + cvt4(u[l + 1], net.Pr[l])
        for B in net.Bpost[l]:
            smooth(l, B)
    z = net.s * vt + conv1(u[0], net.W_out)
    return z.reshape(D.N, D.cells)

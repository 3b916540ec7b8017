"""Each convolution launch of the V-cycle against the oracle's convolutions, element by element.

One launch of `mgnet_conv_apply` (the kernels rte_precond_apply runs, with
their fused epilogues) is compared with oracle.network.conv3 /
conv_transpose4 on the same operands.  On the BF16 path both sides take the
input and the weights rounded to bfloat16 (nearest even): the GPU rounds the
FP32 values it reads, the oracle rounds the same FP32 values with
round_bf16 and sums in FP64.  What is left is FP32 accumulation, so every
element must satisfy

    |gpu - oracle| <= TOL * (sum of |products| + |epilogue terms|)

with TOL = 1e-5: a fixed bound, about 3x the FP32 rounding of a 3456-term
sum accumulated as a random walk (sqrt(3456) * 2^-24 = 3.5e-6) and far below
one bfloat16 step (2^-8), so a wrong tap, channel, pixel or epilogue term
fails it.  Cases cover the 3x3 stride-1 convolution with every epilogue,
the stride-2 restriction, the stride-2 transposed prolongation, 16 to 384
channels, 2D and 3D, grids on and off the tiled kernels' 8- and 4-pixel
patches, and 1, 3 and 32 slots per launch.
"""
import ctypes as C
import zlib

import numpy as np
import pytest

from gpu_util import say, torch_cuda
from oracle import network
from rte_inputs import weights

pytestmark = pytest.mark.gpu

TOL = 1e-5

_models = {}


def _model(dim, c0, levels):
    key = (dim, c0, levels)
    if key not in _models:
        from paper_2604_23265_amd import api
        hdr, t = weights.seeded_weights(dim, 8, c0, levels, 2, 2, 2, 3, seed=900 + c0 + 7 * dim)
        blob = weights.pack_mgn1(hdr, t)
        _models[key] = (api.Model(blob), network.Net(blob))
    return _models[key]


def _weights(net, which, level, index):
    from paper_2604_23265_amd import _lib as L
    if which == L.W_A:
        return net.A[level]
    if which == L.W_BPRE:
        return net.Bpre[level][index]
    if which == L.W_BPOST:
        return net.Bpost[level][index]
    if which == L.W_BCOARSE:
        return net.Bc[index]
    if which == L.W_R:
        return net.R[level]
    return net.Pr[level]


def _to_oracle(a, sp, c):
    """[pixels][c] (x fastest) -> [c, *spatial] with spatial = (ny, nx) or (nz, ny, nx)."""
    return np.moveaxis(a.reshape(tuple(sp) + (c,)), -1, 0)


def _from_oracle(a):
    return np.moveaxis(a, 0, -1).reshape(-1, a.shape[0])


# (dim, c0, levels, level, weights, epilogue, input grid (x, y, z), slots, precision)
W = dict(A=0, BPRE=1, BPOST=2, BC=3, R=4, PR=5)
E = dict(STORE=0, ACCUM=1, STORE_T=2, RESID_R=3, RESID_T=4)
CASES = [
    # 2D, 3x3 stride 1: every epilogue; 16..384 channels; tiled (grids of 8) and generic
    (2, 32, 4, 0, "A", "RESID_T", (16, 16, 1), 1, "bf16"),
    (2, 32, 4, 0, "BPRE", "ACCUM", (16, 16, 1), 3, "bf16"),
    (2, 32, 4, 0, "BPOST", "STORE", (24, 16, 1), 32, "bf16"),
    (2, 32, 4, 0, "A", "RESID_R", (16, 16, 1), 3, "bf16"),
    (2, 32, 4, 1, "A", "RESID_T", (16, 16, 1), 32, "bf16"),
    (2, 32, 4, 2, "BPOST", "ACCUM", (8, 8, 1), 3, "bf16"),
    (2, 32, 4, 3, "BC", "ACCUM", (8, 8, 1), 32, "bf16"),
    (2, 32, 4, 3, "A", "RESID_T", (8, 8, 1), 1, "bf16"),
    (2, 48, 4, 0, "A", "RESID_T", (16, 16, 1), 3, "bf16"),
    (2, 48, 4, 1, "BPRE", "ACCUM", (8, 8, 1), 3, "bf16"),
    (2, 48, 4, 3, "A", "RESID_R", (8, 8, 1), 3, "bf16"),
    (2, 48, 4, 3, "BC", "STORE", (8, 8, 1), 32, "bf16"),
    (2, 16, 4, 0, "A", "RESID_T", (16, 16, 1), 3, "bf16"),
    (2, 16, 4, 0, "BPRE", "ACCUM", (16, 16, 1), 1, "bf16"),
    (2, 16, 4, 2, "A", "RESID_T", (12, 12, 1), 3, "bf16"),
    (2, 32, 4, 0, "A", "RESID_T", (12, 12, 1), 3, "bf16"),
    (2, 32, 4, 1, "BPRE", "ACCUM", (20, 12, 1), 1, "bf16"),
    # 16 x 8 patches (several along x and y) of the wide 3x3 kernel
    (2, 32, 4, 0, "A", "RESID_T", (32, 8, 1), 3, "bf16"),
    (2, 32, 4, 1, "BPOST", "ACCUM", (16, 24, 1), 32, "bf16"),
    (2, 48, 4, 1, "A", "RESID_R", (32, 16, 1), 3, "bf16"),
    (2, 32, 4, 0, "A", "STORE_T", (48, 16, 1), 1, "bf16"),
    # 2D restriction (stride 2) and transposed prolongation
    (2, 32, 4, 0, "R", "STORE_T", (16, 16, 1), 3, "bf16"),
    (2, 32, 4, 0, "R", "STORE", (16, 16, 1), 32, "bf16"),
    (2, 32, 4, 2, "R", "STORE_T", (16, 16, 1), 1, "bf16"),
    (2, 48, 4, 2, "R", "STORE_T", (16, 16, 1), 3, "bf16"),
    (2, 16, 4, 0, "R", "STORE_T", (12, 12, 1), 3, "bf16"),
    (2, 32, 4, 0, "PR", "ACCUM", (8, 8, 1), 3, "bf16"),
    (2, 32, 4, 2, "PR", "STORE", (4, 4, 1), 32, "bf16"),
    (2, 32, 4, 1, "PR", "ACCUM", (8, 8, 1), 1, "bf16"),
    (2, 48, 4, 2, "PR", "ACCUM", (8, 8, 1), 3, "bf16"),
    (2, 16, 4, 0, "PR", "ACCUM", (6, 6, 1), 3, "bf16"),
    # 3D
    (3, 16, 3, 0, "A", "RESID_T", (8, 8, 8), 3, "bf16"),
    (3, 16, 3, 0, "BPRE", "ACCUM", (8, 8, 8), 1, "bf16"),
    (3, 48, 3, 0, "A", "RESID_T", (8, 8, 8), 3, "bf16"),
    (3, 48, 3, 1, "BPOST", "ACCUM", (4, 4, 4), 3, "bf16"),
    (3, 48, 3, 2, "BC", "STORE", (4, 4, 4), 1, "bf16"),
    (3, 16, 3, 0, "A", "RESID_R", (6, 6, 6), 3, "bf16"),
    (3, 48, 3, 0, "R", "STORE_T", (8, 8, 8), 3, "bf16"),
    (3, 48, 3, 0, "PR", "ACCUM", (4, 4, 4), 3, "bf16"),
    (3, 16, 3, 1, "PR", "STORE", (4, 4, 4), 1, "bf16"),
    # the FP32 path
    (2, 32, 4, 0, "A", "RESID_T", (16, 16, 1), 3, "fp32"),
    (2, 32, 4, 1, "BPRE", "ACCUM", (8, 8, 1), 1, "fp32"),
    (2, 32, 4, 0, "R", "STORE_T", (16, 16, 1), 3, "fp32"),
    (2, 32, 4, 0, "PR", "ACCUM", (8, 8, 1), 3, "fp32"),
    (3, 16, 3, 0, "A", "RESID_T", (8, 8, 8), 3, "fp32"),
    (3, 16, 3, 0, "PR", "ACCUM", (4, 4, 4), 1, "fp32"),
]


def _id(c):
    dim, c0, levels, lv, w, e, g, ns, prec = c
    return "%dd-c%d-l%d-%s-%s-%s-s%d-%s" % (dim, c0 << lv, lv, w, e, "x".join(map(str, g[:dim])), ns, prec)


@pytest.mark.parametrize("case", CASES, ids=[_id(c) for c in CASES])
def test_conv_launch_matches_oracle(case):
    torch = torch_cuda()
    from paper_2604_23265_amd import _lib as L
    dim, c0, levels, level, wname, ename, grid, nslots, prec = case
    which, epi = W[wname], E[ename]
    say("conv case", _id(case))
    model, net = _model(dim, c0, levels)
    Wt = _weights(net, which, level, 0)
    if which == W["PR"]:
        cin, cout = Wt.shape[0], Wt.shape[1]
    else:
        cout, cin = Wt.shape[0], Wt.shape[1]
    sp_in = tuple(reversed(grid[:dim]))             # (ny, nx) or (nz, ny, nx)
    if which == W["R"]:
        sp_out = tuple(s // 2 for s in sp_in)
    elif which == W["PR"]:
        sp_out = tuple(2 * s for s in sp_in)
    else:
        sp_out = sp_in
    pin, pout = int(np.prod(sp_in)), int(np.prod(sp_out))
    rng = np.random.default_rng(zlib.crc32(_id(case).encode()))
    x = rng.standard_normal((nslots, pin, cin)).astype(np.float32)
    f = rng.standard_normal((nslots, pout, cout)).astype(np.float32)
    a = rng.uniform(0.2, 2.0, (nslots, pout, cout)).astype(np.float32)
    ai = rng.uniform(0.2, 2.0, (nslots, pout, cout)).astype(np.float32)
    out0 = rng.standard_normal((nslots, pout, cout)).astype(np.float32)

    stride_el = ((max(pin * cin, pout * cout) + 63) // 64) * 64
    def slab(arr):
        buf = np.zeros((nslots, stride_el), np.float32)
        buf[:, :arr.shape[1] * arr.shape[2]] = arr.reshape(nslots, -1)
        return torch.from_numpy(buf).cuda()
    dx, df, da, dai, dout = slab(x), slab(f), slab(a), slab(ai), slab(out0)
    dout2 = torch.zeros_like(dout)
    table = torch.zeros(128 * nslots, dtype=torch.uint8, device="cuda") if nslots > 1 else None
    dims = (C.c_int * 3)(*grid)
    pc = L.PC_MGNET_BF16 if prec == "bf16" else L.PC_MGNET_FP32
    L.check(L.lib().mgnet_conv_apply(model.handle, pc, which, level, 0, epi, dims, nslots, stride_el * 4,
                                     dx.data_ptr(), dout.data_ptr(), dout2.data_ptr(), df.data_ptr(),
                                     da.data_ptr(), dai.data_ptr(),
                                     table.data_ptr() if table is not None else None, None))
    got = dout.cpu().numpy()[:, :pout * cout].reshape(nslots, pout, cout).astype(np.float64)
    got2 = dout2.cpu().numpy()[:, :pout * cout].reshape(nslots, pout, cout).astype(np.float64)

    Wd = Wt if prec == "fp32" else network.round_bf16(Wt)
    worst = 0.0
    for s in range(nslots):
        xo = _to_oracle(x[s].astype(np.float64), sp_in, cin)
        xr = xo if prec == "fp32" else network.round_bf16(xo)
        if which == W["PR"]:
            conv = network.conv_transpose4(xr, Wd)
            mag = network.conv_transpose4(np.abs(xr), np.abs(Wd))
        else:
            st = 2 if which == W["R"] else 1
            conv = network.conv3(xr, Wd, stride=st)
            mag = network.conv3(np.abs(xr), np.abs(Wd), stride=st)
        conv, mag = _from_oracle(conv), _from_oracle(mag)
        fs, as_, ais, o0 = (z[s].astype(np.float64) for z in (f, a, ai, out0))
        u = x[s].astype(np.float64)
        ref2 = None
        if ename == "STORE":
            ref, scale = conv, mag
        elif ename == "ACCUM":
            ref, scale = o0 + conv, np.abs(o0) + mag
        elif ename == "STORE_T":
            ref, scale = conv, mag
            ref2, scale2 = ais * conv, ais * mag
        elif ename == "RESID_R":
            ref, scale = fs - conv - as_ * u, np.abs(fs) + mag + np.abs(as_ * u)
        else:
            ref = ais * (fs - conv - as_ * u)
            scale = ais * (np.abs(fs) + mag + np.abs(as_ * u))
        err = np.abs(got[s] - ref)
        bad = err > TOL * scale + 1e-30
        worst = max(worst, float(np.max(err / (scale + 1e-300))))
        assert not bad.any(), ("slot", s, "elements off", int(bad.sum()), "worst relative", worst)
        if ref2 is not None:
            err2 = np.abs(got2[s] - ref2)
            assert not (err2 > TOL * scale2 + 1e-30).any(), ("slot", s, "out2")
            worst = max(worst, float(np.max(err2 / (scale2 + 1e-300))))
    say("  worst |gpu - oracle| / scale = %.2e" % worst)

// MgNet / CoeffNet kernels (paper Sec. 3.2-3.3).
//
// Activations are channels-last FP32: [pixels][C], pixels ordered x fastest.
// Every convolution is an implicit GEMM: rows are the pixels of a "virtual
// grid" (the output grid, or one parity class of it for the transposed
// convolution), columns are output channels, and the reduction runs over
// taps x input channels.  The BF16 convolutions of the MgNet shapes run in
// the LDS-tiled kernels further down (conv_tile_kernel in 2D,
// conv_tile3_kernel in 3D); the generic kernel described here takes the
// FP32 path and the remaining shapes.  Each wave computes a 16-row x (16 NT)-column
// tile; a 256-thread block holds four such waves, either on four row groups
// or, when the launch would otherwise leave the chip underfilled (coarse
// levels), on one row group with the k-steps split four ways.  Operands are
// read straight from global memory into MFMA fragments -- each lane loads 4
// (or 8) consecutive channels of one pixel (16/32 bytes) and the matching
// input channels of one output channel's weights, which are pre-packed
// [tap][cout][cin] -- with the next k-step's loads issued before the current
// step's MFMAs; reuse of a pixel's channels across output-channel tiles
// happens in registers and reuse across taps in the caches.
//
// MFMA operand layout (16x16 output tile): lane l supplies row (l mod 16)
// of A and column (l mod 16) of B for k-group l/16; it receives D rows
// 4 (l/16) + j, j = 0..3, of column (l mod 16).  A and B agree on which
// physical channel sits in each (k-group, slot), so the channel order inside
// a k-step is free.
//
// Epilogues fuse the smoother's pointwise work:
//   STORE   out = conv
//   ACCUM   out += conv
//   RESID_R out = f - conv - a (.) u           (u = the conv input, same grid)
//   RESID_T out = a^{-1} (.) (f - conv - a (.) u)
//   STORE_T out = conv, out2 = a^{-1} (.) conv
// On the BF16 path the tensors that only ever feed a convolution (t: the
// outputs of RESID_T and RESID_R, out2 of STORE_T, the lift's a^{-1} (.) f)
// can be stored as bfloat16 (the tiled 2D kernel's IN16 / T16 forms): they
// are rounded where they are produced exactly as the consumer would round
// them when staging, so the results are bitwise those of FP32 storage.
#include <algorithm>
#include <type_traits>
#include <cstring>

#include "common.h"
#include "taps.h"

namespace rte {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

struct ConvArgs {
  Slots sl;
  const float* in;
  const void* w;
  float* out;
  float* out2;
  const float* f;
  const float* a;
  const float* ainv;
  int in_dim[3];
  int out_dim[3];
  int g_dim[3];
  int cin, cout, cstride, ostride, ntap, mode;
  int transposed;  // 0: 3-tap cross-correlation, 1: kernel-4 stride-2 transposed
  int dim;
};

__device__ inline short bf16_bits(float v) {
  __bf16 h = __bf16(v);
  return __builtin_bit_cast(short, h);
}

template <int KIND> struct BType;
template <> struct BType<0> { typedef float4 type; typedef float elem; };
template <> struct BType<1> { typedef v4s type; typedef uint16_t elem; };
template <> struct BType<2> { typedef v8bf type; typedef uint16_t elem; };

// Operand registers of one k-step: KPL input channels of this lane's pixel
// and, per output-channel tile, KPL weights of this lane's output channel.
template <int KIND, int NT>
struct Ops {
  float4 a0, a1;
  typename BType<KIND>::type b[NT];
};

// Loads are unconditional (the address is always inside the tensor) and
// out-of-range taps are zeroed with a select afterwards: no branch separates
// the loads of a batch, so none of them waits for the others.
template <int KIND, int NT>
__device__ inline void load_ops(Ops<KIND, NT>& o, const float* ap, bool inb, const void* w, size_t woff,
                                int cin) {
  const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
  const float4 l0 = *reinterpret_cast<const float4*>(ap);
  o.a0 = inb ? l0 : z4;
  if (KIND == 2) {
    const float4 l1 = *reinterpret_cast<const float4*>(ap + 4);
    o.a1 = inb ? l1 : z4;
  } else {
    o.a1 = z4;
  }
  typedef typename BType<KIND>::elem E;
  typedef typename BType<KIND>::type T;
  const E* W = static_cast<const E*>(w) + woff;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) o.b[nt] = *reinterpret_cast<const T*>(W + size_t(nt) * 16 * cin);
}

template <int KIND, int NT>
__device__ inline void mma(v4f* acc, const Ops<KIND, NT>& o) {
  if constexpr (KIND == 0) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a0.x, o.b[nt].x, acc[nt], 0, 0, 0);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a0.y, o.b[nt].y, acc[nt], 0, 0, 0);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a0.z, o.b[nt].z, acc[nt], 0, 0, 0);
      acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a0.w, o.b[nt].w, acc[nt], 0, 0, 0);
    }
  } else if constexpr (KIND == 1) {
    const v4s av = v4s{bf16_bits(o.a0.x), bf16_bits(o.a0.y), bf16_bits(o.a0.z), bf16_bits(o.a0.w)};
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, o.b[nt], acc[nt], 0, 0, 0);
  } else {
    v8bf av;
    av[0] = __bf16(o.a0.x); av[1] = __bf16(o.a0.y); av[2] = __bf16(o.a0.z); av[3] = __bf16(o.a0.w);
    av[4] = __bf16(o.a1.x); av[5] = __bf16(o.a1.y); av[6] = __bf16(o.a1.z); av[7] = __bf16(o.a1.w);
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, o.b[nt], acc[nt], 0, 0, 0);
  }
}

__device__ inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// KSPLIT = false: the block's 4 waves own 4 consecutive 16-row groups and
// run the whole reduction.  KSPLIT = true: the 4 waves share one 16-row
// group and each runs a quarter of the k-steps; waves 1-3 hand their
// partial tiles to wave 0 through LDS, which adds them in wave order
// (deterministic) and writes the epilogue.  The k-loop runs in batches of
// DEPTH k-steps whose operand loads are all issued before the batch's MFMAs;
// the last (< DEPTH) steps run singly.
template <int KIND, int NT, bool KSPLIT, int MODE>
__global__ __launch_bounds__(256) void conv_kernel(const ConvArgs A0) {
  // grid z = slot * classes + parity class of the transposed convolution
  const int nclass = A0.transposed ? (1 << A0.dim) : 1;
  const int slot_z = int(blockIdx.z) / nclass;
  const int cls = int(blockIdx.z) - slot_z * nclass;
  SlotBase bs;
  if (!slot_open(A0.sl, slot_z, bs)) return;
  ConvArgs A = A0;
  A.in = at(A0.in, bs.ws);
  A.out = at(A0.out, bs.ws);
  A.out2 = at(A0.out2, bs.ws);
  A.f = at(A0.f, bs.ws);
  A.a = at(A0.a, bs.op);
  A.ainv = at(A0.ainv, bs.op);
  constexpr int KPL = KIND == 2 ? 8 : 4;  // channels per lane per k-step
  constexpr int KC = 4 * KPL;             // channels per k-step
  const int lane = threadIdx.x & 63;
  // wave-uniform by construction; readfirstlane lets the compiler keep the
  // k-step bookkeeping (tap, channel chunk, tap offsets) in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int grp = lane >> 4, li = lane & 15;
  // row indices fit in 32 bits (pixels per level < 2^31)
  const int gx = A.g_dim[0], gy = A.g_dim[1];
  const int gm = gx * gy * A.g_dim[2];
  const int rbase = KSPLIT ? int(blockIdx.x) * 16 : int(blockIdx.x) * 64 + wave * 16;
  const int co0 = blockIdx.y * (NT * 16);
  const int row = rbase + li;
  const bool rv = row < gm;
  int X, Y, Z;
  {
    const int rc = rv ? row : gm - 1;  // address a valid row; zeroed below
    const int t = rc / gx;
    X = rc - t * gx;
    Z = t / gy;
    Y = t - Z * gy;
  }
  v4f acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = v4f{0.f, 0.f, 0.f, 0.f};

  const int cin = A.cin, cout = A.cout;
  const int nchunk = cin / KC;
  const int nks = A.ntap * nchunk;
  int ks0 = 0, ks1 = nks;
  if (KSPLIT) {
    ks0 = (nks * wave) >> 2;
    ks1 = (nks * (wave + 1)) >> 2;
  }
  int tap = ks0 / nchunk;
  int ci0 = (ks0 - tap * nchunk) * KC;
  // Tap offsets are computed from the (wave-uniform) tap index: a table in
  // memory would be a per-lane load that every k-step has to wait for.
  // Per lane only the base coordinates and a 32-bit element offset vary.
  const int xb = A.cstride * X, yb = A.cstride * Y, zb = A.cstride * Z;
  const int W0 = A.in_dim[0], W1 = A.in_dim[1], W2 = A.in_dim[2];
  const int lane_a = grp * KPL;                       // + pixel * cin + c0
  const int lane_w = li * cin + grp * KPL;            // + (tap * cout + co0) * cin + c0
  auto locate = [&](int tp, int c0, const float*& ap, bool& inb, size_t& woff) {
    const int tt = cls * A.ntap + tp;
    int k3[3], off[3];
    if (A.transposed)
      convT4_tap(A.dim, cls, tp, k3, off);
    else
      conv3_tap(A.dim, tp, k3, off);
    const int ix = xb + off[0], iy = yb + off[1], iz = zb + off[2];
    inb = rv && unsigned(ix) < unsigned(W0) && unsigned(iy) < unsigned(W1) && unsigned(iz) < unsigned(W2);
    const int ipix = (clampi(iz, 0, W2 - 1) * W1 + clampi(iy, 0, W1 - 1)) * W0 + clampi(ix, 0, W0 - 1);
    ap = A.in + (ipix * cin + lane_a + c0);
    woff = size_t((tt * cout + co0) * cin + c0) + lane_w;
  };

  // This lane's output rows are r0 .. r0 + 3.  Epilogue operands do not
  // depend on the reduction: request them now so their latency hides under
  // the k-loop (only the wave that writes the epilogue).
  const int r0 = rbase + grp * 4;
  size_t oidx[4];
  bool ovalid[4];
  {
    const int rc = r0 < gm ? r0 : gm - 1;
    const int t = rc / gx;
    int x = rc - t * gx;
    int z = t / gy;
    int y = t - z * gy;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (j > 0 && r0 + j < gm) {
        if (++x == gx) {
          x = 0;
          if (++y == gy) {
            y = 0;
            ++z;
          }
        }
      }
      ovalid[j] = r0 + j < gm;
      // transposed conv: class cls writes output parity (cls & 1, cls >> 1 & 1, cls >> 2 & 1)
      const int ox = A.ostride * x + (A.transposed ? (cls & 1) : 0);
      const int oy = A.ostride * y + (A.transposed ? (cls >> 1) & 1 : 0);
      const int oz = A.ostride * z + (A.transposed && A.dim == 3 ? (cls >> 2) & 1 : 0);
      oidx[j] = size_t((oz * A.out_dim[1] + oy) * A.out_dim[0] + ox) * cout;
    }
  }
  constexpr bool NEED_F = MODE == CONV_RESID_R || MODE == CONV_RESID_T;
  constexpr bool NEED_I = MODE == CONV_RESID_T || MODE == CONV_STORE_T;
  constexpr bool NEED_U = MODE == CONV_ACCUM || NEED_F;
  float ef[4 * NT], ea[4 * NT], ei[4 * NT], eu[4 * NT];
  if (!KSPLIT || wave == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int q = j * NT + nt;
        const size_t o = oidx[j] + co0 + nt * 16 + li;
        if (NEED_F) {
          ef[q] = A.f[o];
          ea[q] = A.a[o];
        }
        if (NEED_I) ei[q] = A.ainv[o];
        if (NEED_U) eu[q] = MODE == CONV_ACCUM ? A.out[o] : A.in[o];
      }
  }

  // Full batches: all DEPTH steps' operand loads are issued before the
  // batch's MFMAs.  The remaining (< DEPTH) steps run one at a time.
  constexpr int DEPTH = NT >= 4 ? 4 : 8;
  auto advance = [&]() {
    ci0 += KC;
    if (ci0 == cin) {
      ci0 = 0;
      ++tap;
    }
  };
  int ks = ks0;
  for (; ks + DEPTH <= ks1; ks += DEPTH) {
    Ops<KIND, NT> buf[DEPTH];
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) {
      const float* ap;
      bool inb;
      size_t woff;
      locate(tap, ci0, ap, inb, woff);
      load_ops<KIND, NT>(buf[d], ap, inb, A.w, woff, cin);
      advance();
    }
#pragma unroll
    for (int d = 0; d < DEPTH; ++d) mma<KIND, NT>(acc, buf[d]);
  }
  for (; ks < ks1; ++ks) {
    Ops<KIND, NT> one;
    const float* ap;
    bool inb;
    size_t woff;
    locate(tap, ci0, ap, inb, woff);
    load_ops<KIND, NT>(one, ap, inb, A.w, woff, cin);
    advance();
    mma<KIND, NT>(acc, one);
  }

  if constexpr (KSPLIT) {
    __shared__ float red[3][NT][4][64];
    if (wave > 0) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int j = 0; j < 4; ++j) red[wave - 1][nt][j][lane] = acc[nt][j];
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[nt][j] += red[w][nt][j][lane];
  }

#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (!ovalid[j]) continue;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int q = j * NT + nt;
      const size_t o = oidx[j] + co0 + nt * 16 + li;
      const float v = acc[nt][j];
      if constexpr (MODE == CONV_STORE) {
        A.out[o] = v;
      } else if constexpr (MODE == CONV_ACCUM) {
        A.out[o] = eu[q] + v;
      } else if constexpr (MODE == CONV_STORE_T) {
        A.out[o] = v;
        A.out2[o] = ei[q] * v;
      } else if constexpr (MODE == CONV_RESID_R) {
        A.out[o] = ef[q] - v - ea[q] * eu[q];
      } else {
        A.out[o] = ei[q] * (ef[q] - v - ea[q] * eu[q]);
      }
    }
  }
}

// 3x3, stride-1, 2D convolution with the block's input footprint staged in
// LDS (BF16 weights, cin a multiple of 32, grid width a multiple of 16).
// The block owns ROWS consecutive pixels of the row-major grid: a 64- (or
// 16-) pixel segment of one image row, or 64/gx whole rows of a narrow grid.
// Per 32-channel chunk the footprint (rows + halo) is read from global once,
// rounded to BF16 and written to LDS with an 80-byte pixel stride (the 16-
// byte A-fragment reads of eight consecutive lanes then hit distinct banks);
// all 9 taps read their A fragments from LDS.  Chunks are double-buffered.
// KSPLIT: the 4 waves share 16 pixels and split the 9 taps (3, 2, 2, 2);
// their partial tiles are combined in LDS in wave order.
constexpr int LDS_PIX_WORDS = 20;  // 32 BF16 channels (16 words) + 4 words of padding

template <int NT, bool KSPLIT, int MODE>
__global__ __launch_bounds__(256) void conv3_lds_kernel(const ConvArgs A0) {
  SlotBase bs;
  if (!slot_open(A0.sl, int(blockIdx.z), bs)) return;
  ConvArgs A = A0;
  A.in = at(A0.in, bs.ws);
  A.out = at(A0.out, bs.ws);
  A.out2 = at(A0.out2, bs.ws);
  A.f = at(A0.f, bs.ws);
  A.a = at(A0.a, bs.op);
  A.ainv = at(A0.ainv, bs.op);
  constexpr int ROWS = KSPLIT ? 16 : 64;
  constexpr int KC = 32;
  extern __shared__ uint32_t tile[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int grp = lane >> 4, li = lane & 15;
  const int gx = A.g_dim[0], gy = A.g_dim[1];
  const int gm = gx * gy;
  const int cin = A.cin, cout = A.cout;
  const int nchunk = cin / KC;
  const int rb = int(blockIdx.x) * ROWS;
  const int co0 = blockIdx.y * (NT * 16);
  // footprint of the block: rows y0 .. y0 + nrow - 1, columns x0 .. x0 + width - 1
  const int y0 = rb / gx;
  const int x0 = rb - y0 * gx;
  const int width = gx >= ROWS ? ROWS : gx;
  const int nrow = gx >= ROWS ? 1 : ROWS / gx;
  const int TW = width + 2, TH = nrow + 2;
  const int tpix = TW * TH;
  uint32_t* buf[2] = {tile, tile + tpix * LDS_PIX_WORDS};

  // stage chunk c of the footprint into LDS buffer b (all 256 threads)
  auto stage = [&](int c, int b) {
    uint32_t* dst = buf[b];
    const int n4 = tpix * 8;  // float4 pieces: 8 per pixel (32 channels)
    for (int idx = threadIdx.x; idx < n4; idx += 256) {
      const int pix = idx >> 3, c4 = idx & 7;
      const int ty = pix / TW, tx = pix - ty * TW;
      const int iy = y0 - 1 + ty, ix = x0 - 1 + tx;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (unsigned(iy) < unsigned(gy) && unsigned(ix) < unsigned(gx))
        v = *reinterpret_cast<const float4*>(A.in + size_t(iy * gx + ix) * cin + c * KC + c4 * 4);
      const uint32_t lo = uint32_t(uint16_t(bf16_bits(v.x))) | (uint32_t(uint16_t(bf16_bits(v.y))) << 16);
      const uint32_t hi = uint32_t(uint16_t(bf16_bits(v.z))) | (uint32_t(uint16_t(bf16_bits(v.w))) << 16);
      *reinterpret_cast<uint2*>(dst + pix * LDS_PIX_WORDS + c4 * 2) = make_uint2(lo, hi);
    }
  };

  // this lane's A row: pixel rb + (wave's 16-row group) + li
  const int wrow = KSPLIT ? 0 : wave * 16;
  const int r = rb + wrow + li;
  const int ly = (wrow + li) / width, lx = (wrow + li) - ((wrow + li) / width) * width;  // within footprint
  // taps of this wave
  const int t_first = KSPLIT ? wave : 0;
  const int t_step = KSPLIT ? 4 : 1;

  // epilogue rows of this lane: rb + wrow + grp * 4 + j (consecutive pixels of one image row)
  const int r0 = rb + wrow + grp * 4;
  size_t oidx[4];
  bool ovalid[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    ovalid[j] = r0 + j < gm;
    oidx[j] = size_t(ovalid[j] ? r0 + j : 0) * cout;
  }
  constexpr bool NEED_F = MODE == CONV_RESID_R || MODE == CONV_RESID_T;
  constexpr bool NEED_I = MODE == CONV_RESID_T || MODE == CONV_STORE_T;
  constexpr bool NEED_U = MODE == CONV_ACCUM || NEED_F;
  float ef[4 * NT], ea[4 * NT], ei[4 * NT], eu[4 * NT];
  if (!KSPLIT || wave == 0) {
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int q = j * NT + nt;
        const size_t o = oidx[j] + co0 + nt * 16 + li;
        if (NEED_F) {
          ef[q] = A.f[o];
          ea[q] = A.a[o];
        }
        if (NEED_I) ei[q] = A.ainv[o];
        if (NEED_U) eu[q] = MODE == CONV_ACCUM ? A.out[o] : A.in[o];
      }
  }

  v4f acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = v4f{0.f, 0.f, 0.f, 0.f};
  const uint16_t* W = static_cast<const uint16_t*>(A.w);
  const size_t wlane = size_t(co0 + li) * cin + grp * 8;

  stage(0, 0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int b = c & 1;
    if (c + 1 < nchunk) stage(c + 1, b ^ 1);  // next chunk loads while this one computes
    // B fragments of this wave's taps (t = t_first + i t_step) for chunk c
    constexpr int TPW = KSPLIT ? 3 : 9;
    v8bf bw[TPW][NT];
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = t_first + i * t_step;
      if (t >= 9) continue;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        bw[i][nt] = *reinterpret_cast<const v8bf*>(W + (size_t(t) * cout + nt * 16) * cin + wlane + c * KC);
    }
    const uint32_t* src = buf[b];
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = t_first + i * t_step;
      if (t >= 9) continue;
      const int ky = t / 3, kx = t - (t / 3) * 3;
      const int pix = (ly + ky) * TW + (lx + kx);
      const v8bf av = *reinterpret_cast<const v8bf*>(src + pix * LDS_PIX_WORDS + grp * 4);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bw[i][nt], acc[nt], 0, 0, 0);
    }
    __syncthreads();  // buffer b is rewritten two chunks later; chunk c + 1 is now complete
  }
  (void)r;

  if constexpr (KSPLIT) {
    float* red = reinterpret_cast<float*>(tile);  // reuse the staging area
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (wave > 0) red[((wave - 1) * NT * 4 + nt * 4 + j) * 64 + lane] = acc[nt][j];
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[nt][j] += red[(w * NT * 4 + nt * 4 + j) * 64 + lane];
  }

#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (!ovalid[j]) continue;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int q = j * NT + nt;
      const size_t o = oidx[j] + co0 + nt * 16 + li;
      const float v = acc[nt][j];
      if constexpr (MODE == CONV_STORE) {
        A.out[o] = v;
      } else if constexpr (MODE == CONV_ACCUM) {
        A.out[o] = eu[q] + v;
      } else if constexpr (MODE == CONV_STORE_T) {
        A.out[o] = v;
        A.out2[o] = ei[q] * v;
      } else if constexpr (MODE == CONV_RESID_R) {
        A.out[o] = ef[q] - v - ea[q] * eu[q];
      } else {
        A.out[o] = ei[q] * (ef[q] - v - ea[q] * eu[q]);
      }
    }
  }
}

// Tiled 2D BF16 convolution: one block computes an 8x8 patch of the
// virtual grid for 32 or 64 output channels.  Per 32-channel input chunk
// the block stages the patch's input footprint (rounded to BF16) and the
// chunk's weights for its output channels in LDS, both in swizzled 64-byte
// rows; while the chunk's MFMAs run, the next chunk's global loads are
// already in flight in registers.  Wave w owns patch rows 2w and 2w + 1
// (16 pixels) and every 16-channel column tile.
//
// CK = 0: 3x3 stride 1; CK = 1: 3x3 stride 2 (restriction); CK = 2: the
// 4x4 stride-2 transposed convolution, one parity class per grid-z index.
// Every output element accumulates its chunks in order and, within a chunk,
// its taps in order -- the same chain whatever the launch shape, so results
// do not depend on how many solves share the launch.
// LDS rows of the tiled conv: 32 BF16 (64 bytes, four 16-byte chunks), no
// padding; chunk q of row r sits at chunk q ^ ((r >> 1) & 3).  Measured on
// gfx950 with the bank-conflict counter, this order makes the 16-byte
// fragment reads of the weights and both staging stores conflict-free (an
// 80-byte padded row spends half of its LDS cycles in conflicts).
constexpr int TILE_ROW_WORDS = 16;
__device__ inline int tile_word(int row, int chunk) { return row * TILE_ROW_WORDS + 4 * (chunk ^ ((row >> 1) & 3)); }
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

template <int CK, int NI>
struct TileGeom {
  static constexpr int NTAP = CK == 2 ? 4 : 9;
  static constexpr int S = CK == 1 ? 2 : 1;                       // input step per virtual pixel
  static constexpr int FP = CK == 0 ? 10 : (CK == 1 ? 17 : 9);    // footprint extent per axis
  static constexpr int FPIX = FP * FP;
  static constexpr int NCLS = CK == 2 ? 4 : 1;
  static constexpr int NCO = 16 * NI;                             // output channels per block
  static constexpr int IN_PIECES = (FPIX * 8 + 255) / 256;        // float4 loads per thread
  static constexpr int W_PIECES = (NTAP * NCO * 4 + 255) / 256;   // 16-byte weight loads per thread
};

// NI = 2 or 4 column tiles of 16 output channels per block (32 or 64
// channels): with 64 the input footprint is staged once per 64 outputs.
template <int CK, int MODE, int NI, bool IN16, bool T16>
__global__ __launch_bounds__(256) void conv_tile_kernel(const ConvArgs A0) {
  using G = TileGeom<CK, NI>;
  static_assert(!IN16 || MODE == CONV_STORE || MODE == CONV_ACCUM || MODE == CONV_STORE_T,
                "a BF16 input is a t tensor, never the u of a residual epilogue");
  static_assert(!T16 || MODE == CONV_RESID_T || MODE == CONV_RESID_R || MODE == CONV_STORE_T,
                "only t outputs are stored as BF16");
  // the footprint of one 32-channel chunk: 8 float4 per pixel, or 4 pieces
  // of 8 BF16
  constexpr int PIECES_PER_PIX = IN16 ? 4 : 8;
  constexpr int INP = (G::FPIX * PIECES_PER_PIX + 255) / 256;
  const int slot_z = int(blockIdx.z) / G::NCLS;
  const int cls = int(blockIdx.z) - slot_z * G::NCLS;
  SlotBase bs;
  if (!slot_open(A0.sl, slot_z, bs)) return;
  const float* __restrict__ in = at(A0.in, bs.ws);
  float* __restrict__ out = at(A0.out, bs.ws);
  float* __restrict__ out2 = at(A0.out2, bs.ws);
  const float* __restrict__ fF = at(A0.f, bs.ws);
  const float* __restrict__ fA = at(A0.a, bs.op);
  const float* __restrict__ fI = at(A0.ainv, bs.op);
  const uint16_t* __restrict__ W = static_cast<const uint16_t*>(A0.w);

  __shared__ uint32_t xin[G::FPIX * TILE_ROW_WORDS];
  __shared__ uint32_t wsm[G::NTAP * G::NCO * TILE_ROW_WORDS];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int grp = lane >> 4, li = lane & 15;
  const int gx = A0.g_dim[0];
  const int npx = gx >> 3;
  const int patch = blockIdx.x;
  const int py0 = (patch / npx) * 8, px0 = (patch - (patch / npx) * npx) * 8;
  const int co0 = blockIdx.y * G::NCO;
  const int W0 = A0.in_dim[0], W1 = A0.in_dim[1];
  const int cin = A0.cin, cout = A0.cout;
  const int nchunk = cin >> 5;
  const int px_par = cls & 1, py_par = (cls >> 1) & 1;
  // input coordinates of footprint entry (0, 0)
  const int ox0 = CK == 1 ? 2 * px0 - 1 : (CK == 2 ? px0 - 1 + px_par : px0 - 1);
  const int oy0 = CK == 1 ? 2 * py0 - 1 : (CK == 2 ? py0 - 1 + py_par : py0 - 1);

  // ---- epilogue operands (independent of the reduction): request them now
  const int ox_dim = A0.out_dim[0];
  size_t oidx[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int pr = 4 * grp + j;  // D row -> patch pixel (pr % 8, 2 wave + pr / 8)
    const int vx = px0 + (pr & 7), vy = py0 + 2 * wave + (pr >> 3);
    const int ox = CK == 2 ? 2 * vx + px_par : vx;
    const int oy = CK == 2 ? 2 * vy + py_par : vy;
    oidx[j] = size_t(oy * ox_dim + ox) * cout + co0 + li;
  }
  constexpr bool NEED_F = MODE == CONV_RESID_R || MODE == CONV_RESID_T;
  constexpr bool NEED_I = MODE == CONV_RESID_T || MODE == CONV_STORE_T;
  constexpr bool NEED_U = MODE == CONV_ACCUM || NEED_F;
  float ef[4 * NI], ea[4 * NI], ei[4 * NI], eu[4 * NI];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      const int q = j * NI + ni;
      const size_t o = oidx[j] + ni * 16;
      if (NEED_F) {
        ef[q] = fF[o];
        ea[q] = fA[o];
      }
      if (NEED_I) ei[q] = fI[o];
      if (NEED_U) eu[q] = MODE == CONV_ACCUM ? out[o] : in[o];
    }

  // ---- staging: chunk c's footprint and weights, loaded into registers
  const uint16_t* __restrict__ in16 = reinterpret_cast<const uint16_t*>(in);
  v4f rin[IN16 ? 1 : INP];
  v4u rin16[IN16 ? INP : 1];
  v4u rw[G::W_PIECES];
  auto load_chunk = [&](int c) {
#pragma unroll
    for (int i = 0; i < INP; ++i) {
      const int idx = int(threadIdx.x) + 256 * i;
      const int pix = idx / PIECES_PER_PIX, qp = idx - (idx / PIECES_PER_PIX) * PIECES_PER_PIX;
      const int fy = pix / G::FP, fx = pix - (pix / G::FP) * G::FP;
      const int ix = ox0 + fx, iy = oy0 + fy;
      const bool ok = idx < G::FPIX * PIECES_PER_PIX && unsigned(ix) < unsigned(W0) && unsigned(iy) < unsigned(W1);
      const int ixc = clampi(ix, 0, W0 - 1), iyc = clampi(iy, 0, W1 - 1);
      if constexpr (IN16) {
        const v4u v = *reinterpret_cast<const v4u*>(in16 + size_t(iyc * W0 + ixc) * cin + c * 32 + qp * 8);
        rin16[i] = ok ? v : v4u{0u, 0u, 0u, 0u};
      } else {
        const v4f v = *reinterpret_cast<const v4f*>(in + size_t(iyc * W0 + ixc) * cin + c * 32 + qp * 4);
        rin[i] = ok ? v : v4f{0.f, 0.f, 0.f, 0.f};
      }
    }
#pragma unroll
    for (int i = 0; i < G::W_PIECES; ++i) {
      const int idx = int(threadIdx.x) + 256 * i;
      constexpr int PER_TAP = G::NCO * 4;
      const int idc = idx < G::NTAP * PER_TAP ? idx : G::NTAP * PER_TAP - 1;
      const int t = idc / PER_TAP, rem = idc - (idc / PER_TAP) * PER_TAP, co = rem >> 2, q8 = rem & 3;
      rw[i] = *reinterpret_cast<const v4u*>(
          W + (size_t((cls * G::NTAP + t) * cout + co0 + co)) * cin + c * 32 + q8 * 8);
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int i = 0; i < INP; ++i) {
      const int idx = int(threadIdx.x) + 256 * i;
      if (idx < G::FPIX * PIECES_PER_PIX) {
        if constexpr (IN16) {
          const int pix = idx >> 2, q = idx & 3;
          *reinterpret_cast<v4u*>(xin + tile_word(pix, q)) = rin16[i];
        } else {
          const int pix = idx >> 3, q4 = idx & 7;
          const v4f v = rin[i];
          const uint32_t lo = uint32_t(uint16_t(bf16_bits(v[0]))) | (uint32_t(uint16_t(bf16_bits(v[1]))) << 16);
          const uint32_t hi = uint32_t(uint16_t(bf16_bits(v[2]))) | (uint32_t(uint16_t(bf16_bits(v[3]))) << 16);
          *reinterpret_cast<uint2*>(xin + tile_word(pix, q4 >> 1) + 2 * (q4 & 1)) = make_uint2(lo, hi);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < G::W_PIECES; ++i) {
      const int idx = int(threadIdx.x) + 256 * i;
      constexpr int PER_TAP = G::NCO * 4;
      if (idx < G::NTAP * PER_TAP) {
        const int t = idx / PER_TAP, rem = idx - (idx / PER_TAP) * PER_TAP, co = rem >> 2, q8 = rem & 3;
        *reinterpret_cast<v4u*>(wsm + tile_word(t * G::NCO + co, q8)) = rw[i];
      }
    }
  };

  // this lane's A pixel: patch (li % 8, 2 wave + li / 8)
  const int lx = li & 7, ly = 2 * wave + (li >> 3);
  v4f acc[NI];
#pragma unroll
  for (int ni = 0; ni < NI; ++ni) acc[ni] = v4f{0.f, 0.f, 0.f, 0.f};
  load_chunk(0);
  for (int c = 0; c < nchunk; ++c) {
    if (c > 0) __syncthreads();  // the previous chunk's reads are done
    store_chunk();
    __syncthreads();
    if (c + 1 < nchunk) load_chunk(c + 1);  // in flight during this chunk's MFMAs
#pragma unroll
    for (int t = 0; t < G::NTAP; ++t) {
      // tap offsets (the tables of taps.h, written out for two axes): a 3x3
      // tap t reads (t % 3 - 1, t / 3 - 1); transposed-conv tap t of parity
      // class (px, py) reads (px - t % 2, py - t / 2)
      const int dx = CK == 2 ? px_par - (t & 1) : t % 3 - 1;
      const int dy = CK == 2 ? py_par - (t >> 1) : t / 3 - 1;
      const int fx = G::S * (px0 + lx) + dx - ox0;
      const int fy = G::S * (py0 + ly) + dy - oy0;
      const v8bf av = *reinterpret_cast<const v8bf*>(xin + tile_word(fy * G::FP + fx, grp));
#pragma unroll
      for (int ni = 0; ni < NI; ++ni) {
        const v8bf bv = *reinterpret_cast<const v8bf*>(wsm + tile_word(t * G::NCO + ni * 16 + li, grp));
        acc[ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[ni], 0, 0, 0);
      }
    }
  }

#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      const int q = j * NI + ni;
      const size_t o = oidx[j] + ni * 16;
      const float v = acc[ni][j];
      // a t output stored as BF16 holds the bits the consumer's staging would make
      auto put_t = [&](float* dst, float x) {
        if constexpr (T16)
          reinterpret_cast<uint16_t*>(dst)[o] = uint16_t(bf16_bits(x));
        else
          dst[o] = x;
      };
      if constexpr (MODE == CONV_STORE) {
        out[o] = v;
      } else if constexpr (MODE == CONV_ACCUM) {
        out[o] = eu[q] + v;
      } else if constexpr (MODE == CONV_STORE_T) {
        out[o] = v;
        put_t(out2, ei[q] * v);
      } else if constexpr (MODE == CONV_RESID_R) {
        put_t(out, ef[q] - v - ea[q] * eu[q]);
      } else {
        put_t(out, ei[q] * (ef[q] - v - ea[q] * eu[q]));
      }
    }
}

// Tiled 3D BF16 convolution: one block computes a 4x4x4 patch of the
// virtual grid for 16 NI output channels; wave w owns z-layer w of the
// patch (16 pixels, one MFMA row tile) and all NI column tiles, so each
// input fragment read from LDS feeds NI MFMAs.  Per 32-channel input chunk
// the block stages the patch's input footprint (6^3 pixels for the 3x3x3
// convolution, 5^3 for one parity class of the 4x4x4 transposed one) in the
// same swizzled 64-byte LDS rows as the 2D kernel; the weights are staged
// in rounds of TR taps (one kz-slice of the 3x3x3 kernel when the block has
// more than 16 output channels, else all 27 taps; all 8 taps of the
// transposed one), the next round's loads in flight during the current
// round's MFMAs.  The epilogue operands are read after the reduction: held
// through it, their 4 NI registers per operand cost more occupancy than
// their latency costs once per block.  Channel counts only need to be multiples of 16: a last
// chunk with 16 channels runs the K = 16 MFMA on the first half of each
// row (the other half is staged as zeros and never read).
//
// CK = 0: 3x3x3 stride 1; CK = 2: 4x4x4 stride-2 transposed, one parity
// class per grid-z index (class = px + 2 py + 4 pz, tap = tx + 2 ty + 4 tz,
// the order of the packed weights).  Accumulation runs chunk by chunk and
// tap by tap, independent of the launch shape.
template <int CK, int NI>
struct Tile3Geom {
  static constexpr int NTAP = CK == 2 ? 8 : 27;
  static constexpr int TR = CK == 2 ? 8 : (NI == 1 ? 27 : 9);  // taps per weight round
  static constexpr int NR = NTAP / TR;
  static constexpr int FP = CK == 0 ? 6 : 5;
  static constexpr int FPIX = FP * FP * FP;
  static constexpr int NCLS = CK == 2 ? 8 : 1;
  static constexpr int NCO = 16 * NI;
  static constexpr int IN_PIECES = (FPIX * 8 + 255) / 256;
  static constexpr int W_PIECES = (TR * NCO * 4 + 255) / 256;
};

template <int CK, int MODE, int NI>
__global__ __launch_bounds__(256) void conv_tile3_kernel(const ConvArgs A0) {
  using G = Tile3Geom<CK, NI>;
  const int slot_z = int(blockIdx.z) / G::NCLS;
  const int cls = int(blockIdx.z) - slot_z * G::NCLS;
  SlotBase bs;
  if (!slot_open(A0.sl, slot_z, bs)) return;
  const float* __restrict__ in = at(A0.in, bs.ws);
  float* __restrict__ out = at(A0.out, bs.ws);
  float* __restrict__ out2 = at(A0.out2, bs.ws);
  const float* __restrict__ fF = at(A0.f, bs.ws);
  const float* __restrict__ fA = at(A0.a, bs.op);
  const float* __restrict__ fI = at(A0.ainv, bs.op);
  const uint16_t* __restrict__ W = static_cast<const uint16_t*>(A0.w);

  __shared__ uint32_t xin[G::FPIX * TILE_ROW_WORDS];
  __shared__ uint32_t wsm[G::TR * G::NCO * TILE_ROW_WORDS];

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int grp = lane >> 4, li = lane & 15;
  const int npx = A0.g_dim[0] >> 2, npy = A0.g_dim[1] >> 2;
  const int patch = blockIdx.x;
  const int pxi = patch % npx, pr_ = patch / npx;
  const int px0 = 4 * pxi, py0 = 4 * (pr_ % npy), pz0 = 4 * (pr_ / npy);
  const int co0 = blockIdx.y * G::NCO;
  const int W0 = A0.in_dim[0], W1 = A0.in_dim[1], W2 = A0.in_dim[2];
  const int cin = A0.cin, cout = A0.cout;
  const int nchunk = (cin + 31) >> 5;
  const int px_par = cls & 1, py_par = (cls >> 1) & 1, pz_par = (cls >> 2) & 1;
  // input coordinates of footprint entry (0, 0, 0)
  const int ox0 = CK == 2 ? px0 - 1 + px_par : px0 - 1;
  const int oy0 = CK == 2 ? py0 - 1 + py_par : py0 - 1;
  const int oz0 = CK == 2 ? pz0 - 1 + pz_par : pz0 - 1;

  // ---- output (and epilogue operand) offsets of this lane's D rows
  const int ox_dim = A0.out_dim[0], oy_dim = A0.out_dim[1];
  size_t oidx[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int pr = 4 * grp + j;  // D row -> pixel (pr % 4, pr / 4) of z-layer `wave`
    const int vx = px0 + (pr & 3), vy = py0 + (pr >> 2), vz = pz0 + wave;
    const int ox = CK == 2 ? 2 * vx + px_par : vx;
    const int oy = CK == 2 ? 2 * vy + py_par : vy;
    const int oz = CK == 2 ? 2 * vz + pz_par : vz;
    oidx[j] = (size_t(oz * oy_dim + oy) * ox_dim + ox) * cout + co0 + li;
  }
  // ---- staging into registers: chunk c's footprint, and round r's weights
  // (taps r TR .. r TR + TR - 1) of chunk c; channels at or beyond cin are
  // read at a valid address and zeroed
  v4f rin[G::IN_PIECES];
  v4u rw[G::W_PIECES];
  auto load_in = [&](int c) {
#pragma unroll
    for (int i = 0; i < G::IN_PIECES; ++i) {
      const int idx = int(threadIdx.x) + 256 * i;
      const int pix = idx >> 3, q4 = idx & 7;
      const int fx = pix % G::FP, fyz = pix / G::FP;
      const int fy = fyz % G::FP, fz = fyz / G::FP;
      const int ix = ox0 + fx, iy = oy0 + fy, iz = oz0 + fz;
      const int ch = c * 32 + q4 * 4;
      const bool ok = idx < G::FPIX * 8 && unsigned(ix) < unsigned(W0) && unsigned(iy) < unsigned(W1) &&
                      unsigned(iz) < unsigned(W2) && ch < cin;
      const int ixc = clampi(ix, 0, W0 - 1), iyc = clampi(iy, 0, W1 - 1), izc = clampi(iz, 0, W2 - 1);
      const int chc = ch < cin ? ch : cin - 4;
      const v4f v = *reinterpret_cast<const v4f*>(in + (size_t(izc * W1 + iyc) * W0 + ixc) * cin + chc);
      rin[i] = ok ? v : v4f{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto load_w = [&](int c, int r) {
#pragma unroll
    for (int i = 0; i < G::W_PIECES; ++i) {
      const int idx = int(threadIdx.x) + 256 * i;
      constexpr int PER_TAP = G::NCO * 4;
      const int idc = idx < G::TR * PER_TAP ? idx : G::TR * PER_TAP - 1;
      const int t = idc / PER_TAP, rem = idc - (idc / PER_TAP) * PER_TAP, co = rem >> 2, q8 = rem & 3;
      const int ch = c * 32 + q8 * 8;
      const v4u v = *reinterpret_cast<const v4u*>(
          W + (size_t((cls * G::NTAP + r * G::TR + t) * cout + co0 + co)) * cin + (ch < cin ? ch : cin - 8));
      rw[i] = ch < cin ? v : v4u{0u, 0u, 0u, 0u};
    }
  };
  auto store_in = [&]() {
#pragma unroll
    for (int i = 0; i < G::IN_PIECES; ++i) {
      const int idx = int(threadIdx.x) + 256 * i;
      if (idx < G::FPIX * 8) {
        const int pix = idx >> 3, q4 = idx & 7;
        const v4f v = rin[i];
        const uint32_t lo = uint32_t(uint16_t(bf16_bits(v[0]))) | (uint32_t(uint16_t(bf16_bits(v[1]))) << 16);
        const uint32_t hi = uint32_t(uint16_t(bf16_bits(v[2]))) | (uint32_t(uint16_t(bf16_bits(v[3]))) << 16);
        *reinterpret_cast<uint2*>(xin + tile_word(pix, q4 >> 1) + 2 * (q4 & 1)) = make_uint2(lo, hi);
      }
    }
  };
  auto store_w = [&]() {
#pragma unroll
    for (int i = 0; i < G::W_PIECES; ++i) {
      const int idx = int(threadIdx.x) + 256 * i;
      constexpr int PER_TAP = G::NCO * 4;
      if (idx < G::TR * PER_TAP) {
        const int t = idx / PER_TAP, rem = idx - (idx / PER_TAP) * PER_TAP, co = rem >> 2, q8 = rem & 3;
        *reinterpret_cast<v4u*>(wsm + tile_word(t * G::NCO + co, q8)) = rw[i];
      }
    }
  };

  // this lane's A pixel: (li % 4, li / 4) of z-layer `wave`
  const int lx = li & 3, ly = li >> 2, lz = wave;
  // weight rows t NCO + 16 ni + li: NCO and 16 are multiples of 8, so the
  // swizzle depends on li only and the row offset is a constant per (t, ni)
  const int bfull = tile_word(li, grp), bhalf = tile_word(li, grp >> 1) + 2 * (grp & 1);
  v4f acc[NI];
#pragma unroll
  for (int ni = 0; ni < NI; ++ni) acc[ni] = v4f{0.f, 0.f, 0.f, 0.f};
  load_in(0);
  load_w(0, 0);
  for (int c = 0; c < nchunk; ++c) {
    const bool half = cin - 32 * c == 16;  // uniform: a 16-channel last chunk
    for (int r = 0; r < G::NR; ++r) {
      if (c > 0 || r > 0) __syncthreads();  // the previous round's reads are done
      if (r == 0) store_in();
      store_w();
      __syncthreads();
      // the next round's loads, in flight during this round's MFMAs
      if (r + 1 < G::NR) {
        load_w(c, r + 1);
      } else if (c + 1 < nchunk) {
        load_in(c + 1);
        load_w(c + 1, 0);
      }
#pragma unroll
      for (int t = 0; t < G::TR; ++t) {
        // a 3x3x3 tap u = r TR + t reads (u % 3 - 1, u / 3 % 3 - 1, u / 9 - 1);
        // transposed tap t of class (px, py, pz) reads (px - t % 2, py - t / 2 % 2, pz - t / 4)
        const int u = r * G::TR + t;
        const int dx = CK == 2 ? px_par - (t & 1) : t % 3 - 1;
        const int dy = CK == 2 ? py_par - ((t >> 1) & 1) : (u / 3) % 3 - 1;
        const int dz = CK == 2 ? pz_par - (t >> 2) : u / 9 - 1;
        const int fx = px0 + lx + dx - ox0;
        const int fy = py0 + ly + dy - oy0;
        const int fz = pz0 + lz + dz - oz0;
        const int arow = (fz * G::FP + fy) * G::FP + fx;
        if (half) {
          // K = 16: k-group grp holds channels 4 grp .. 4 grp + 3 of the chunk
          const v4s av = *reinterpret_cast<const v4s*>(xin + tile_word(arow, grp >> 1) + 2 * (grp & 1));
#pragma unroll
          for (int ni = 0; ni < NI; ++ni) {
            const v4s bv = *reinterpret_cast<const v4s*>(wsm + bhalf + (t * G::NCO + ni * 16) * TILE_ROW_WORDS);
            acc[ni] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[ni], 0, 0, 0);
          }
        } else {
          const v8bf av = *reinterpret_cast<const v8bf*>(xin + tile_word(arow, grp));
#pragma unroll
          for (int ni = 0; ni < NI; ++ni) {
            const v8bf bv = *reinterpret_cast<const v8bf*>(wsm + bfull + (t * G::NCO + ni * 16) * TILE_ROW_WORDS);
            acc[ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[ni], 0, 0, 0);
          }
        }
      }
    }
  }

  constexpr bool NEED_F = MODE == CONV_RESID_R || MODE == CONV_RESID_T;
  constexpr bool NEED_I = MODE == CONV_RESID_T || MODE == CONV_STORE_T;
  constexpr bool NEED_U = MODE == CONV_ACCUM || NEED_F;
  float ef[4 * NI], ea[4 * NI], ei[4 * NI], eu[4 * NI];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      const int q = j * NI + ni;
      const size_t o = oidx[j] + ni * 16;
      if (NEED_F) {
        ef[q] = fF[o];
        ea[q] = fA[o];
      }
      if (NEED_I) ei[q] = fI[o];
      if (NEED_U) eu[q] = MODE == CONV_ACCUM ? out[o] : in[o];
    }

#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int ni = 0; ni < NI; ++ni) {
      const int q = j * NI + ni;
      const size_t o = oidx[j] + ni * 16;
      const float v = acc[ni][j];
      if constexpr (MODE == CONV_STORE) {
        out[o] = v;
      } else if constexpr (MODE == CONV_ACCUM) {
        out[o] = eu[q] + v;
      } else if constexpr (MODE == CONV_STORE_T) {
        out[o] = v;
        out2[o] = ei[q] * v;
      } else if constexpr (MODE == CONV_RESID_R) {
        out[o] = ef[q] - v - ea[q] * eu[q];
      } else {
        out[o] = ei[q] * (ef[q] - v - ea[q] * eu[q]);
      }
    }
}

template <int CK, int NI>
void tile3_dispatch2(const ConvArgs& a, dim3 grid, int mode, hipStream_t s, const ProfScope& ps) {
  switch (mode) {
    case CONV_STORE: launch_k(conv_tile3_kernel<CK, CONV_STORE, NI>, grid, dim3(256), 0, s, ps, a); break;
    case CONV_ACCUM: launch_k(conv_tile3_kernel<CK, CONV_ACCUM, NI>, grid, dim3(256), 0, s, ps, a); break;
    case CONV_STORE_T: launch_k(conv_tile3_kernel<CK, CONV_STORE_T, NI>, grid, dim3(256), 0, s, ps, a); break;
    case CONV_RESID_R: launch_k(conv_tile3_kernel<CK, CONV_RESID_R, NI>, grid, dim3(256), 0, s, ps, a); break;
    default: launch_k(conv_tile3_kernel<CK, CONV_RESID_T, NI>, grid, dim3(256), 0, s, ps, a); break;
  }
}

// Output channels per block: the widest of 64 / 48 / 32 / 16 that divides
// cout and still gives at least 1024 blocks (4 per CU), else 16.
template <int CK>
void tile3_dispatch(const ConvArgs& a, int nz, int mode, hipStream_t s, const ProfScope& ps) {
  const int64_t patches = int64_t(a.g_dim[0] / 4) * (a.g_dim[1] / 4) * (a.g_dim[2] / 4);
  int ni = 1;
  for (int cand : {4, 3, 2})
    if (a.cout % (16 * cand) == 0 && patches * (a.cout / (16 * cand)) * nz >= 1024) {
      ni = cand;
      break;
    }
  const dim3 grid(unsigned(patches), unsigned(a.cout / (16 * ni)), unsigned(nz));
  switch (ni) {
    case 4: tile3_dispatch2<CK, 4>(a, grid, mode, s, ps); break;
    case 3: tile3_dispatch2<CK, 3>(a, grid, mode, s, ps); break;
    case 2: tile3_dispatch2<CK, 2>(a, grid, mode, s, ps); break;
    default: tile3_dispatch2<CK, 1>(a, grid, mode, s, ps); break;
  }
}

template <int CK, int NI>
void tile_dispatch2(const ConvArgs& a, dim3 grid, int mode, bool in16, bool t16, hipStream_t s,
                    const ProfScope& ps) {
  auto go = [&](auto kern) { launch_k(kern, grid, dim3(256), 0, s, ps, a); };
  if constexpr (CK == 2) {  // the prolongation reads u and writes u: FP32 only
    switch (mode) {
      case CONV_STORE: go(conv_tile_kernel<CK, CONV_STORE, NI, false, false>); break;
      case CONV_ACCUM: go(conv_tile_kernel<CK, CONV_ACCUM, NI, false, false>); break;
      case CONV_STORE_T: go(conv_tile_kernel<CK, CONV_STORE_T, NI, false, false>); break;
      case CONV_RESID_R: go(conv_tile_kernel<CK, CONV_RESID_R, NI, false, false>); break;
      default: go(conv_tile_kernel<CK, CONV_RESID_T, NI, false, false>); break;
    }
    return;
  } else {
    switch (mode) {
      case CONV_STORE:
        if (in16) go(conv_tile_kernel<CK, CONV_STORE, NI, true, false>);
        else go(conv_tile_kernel<CK, CONV_STORE, NI, false, false>);
        break;
      case CONV_ACCUM:
        if (in16) go(conv_tile_kernel<CK, CONV_ACCUM, NI, true, false>);
        else go(conv_tile_kernel<CK, CONV_ACCUM, NI, false, false>);
        break;
      case CONV_STORE_T:
        if (in16 && t16) go(conv_tile_kernel<CK, CONV_STORE_T, NI, true, true>);
        else if (in16) go(conv_tile_kernel<CK, CONV_STORE_T, NI, true, false>);
        else if (t16) go(conv_tile_kernel<CK, CONV_STORE_T, NI, false, true>);
        else go(conv_tile_kernel<CK, CONV_STORE_T, NI, false, false>);
        break;
      case CONV_RESID_R:
        if (t16) go(conv_tile_kernel<CK, CONV_RESID_R, NI, false, true>);
        else go(conv_tile_kernel<CK, CONV_RESID_R, NI, false, false>);
        break;
      default:
        if (t16) go(conv_tile_kernel<CK, CONV_RESID_T, NI, false, true>);
        else go(conv_tile_kernel<CK, CONV_RESID_T, NI, false, false>);
        break;
    }
  }
}

template <int CK>
void tile_dispatch(const ConvArgs& a, int gx, int gy, int nz, int mode, bool in16, bool t16, hipStream_t s,
                   const ProfScope& ps) {
  const unsigned patches = unsigned((gx / 8) * (gy / 8));
  if (a.cout % 64 == 0)
    tile_dispatch2<CK, 4>(a, dim3(patches, unsigned(a.cout / 64), unsigned(nz)), mode, in16, t16, s, ps);
  else
    tile_dispatch2<CK, 2>(a, dim3(patches, unsigned(a.cout / 32), unsigned(nz)), mode, in16, t16, s, ps);
}

template <bool KSPLIT, int MODE>
void lds_dispatch3(const ConvArgs& a, dim3 grid, int nt, size_t lds, hipStream_t s, const ProfScope& ps) {
  switch (nt) {
    case 4: launch_k(conv3_lds_kernel<4, KSPLIT, MODE>, grid, dim3(256), uint32_t(lds), s, ps, a); break;
    case 2: launch_k(conv3_lds_kernel<2, KSPLIT, MODE>, grid, dim3(256), uint32_t(lds), s, ps, a); break;
    default: launch_k(conv3_lds_kernel<1, KSPLIT, MODE>, grid, dim3(256), uint32_t(lds), s, ps, a); break;
  }
}

template <bool KSPLIT>
void lds_dispatch2(const ConvArgs& a, dim3 grid, int nt, size_t lds, hipStream_t s, const ProfScope& ps) {
  switch (a.mode) {
    case CONV_STORE: lds_dispatch3<KSPLIT, CONV_STORE>(a, grid, nt, lds, s, ps); break;
    case CONV_ACCUM: lds_dispatch3<KSPLIT, CONV_ACCUM>(a, grid, nt, lds, s, ps); break;
    case CONV_STORE_T: lds_dispatch3<KSPLIT, CONV_STORE_T>(a, grid, nt, lds, s, ps); break;
    case CONV_RESID_R: lds_dispatch3<KSPLIT, CONV_RESID_R>(a, grid, nt, lds, s, ps); break;
    default: lds_dispatch3<KSPLIT, CONV_RESID_T>(a, grid, nt, lds, s, ps); break;
  }
}

template <int KIND, bool KSPLIT, int MODE>
void conv_dispatch3(const ConvArgs& a, dim3 grid, int nt, hipStream_t s, const ProfScope& ps) {
  switch (nt) {
    case 4: launch_k(conv_kernel<KIND, 4, KSPLIT, MODE>, grid, dim3(256), 0, s, ps, a); break;
    case 2: launch_k(conv_kernel<KIND, 2, KSPLIT, MODE>, grid, dim3(256), 0, s, ps, a); break;
    default: launch_k(conv_kernel<KIND, 1, KSPLIT, MODE>, grid, dim3(256), 0, s, ps, a); break;
  }
}

template <int KIND, bool KSPLIT>
void conv_dispatch2(const ConvArgs& a, dim3 grid, int nt, hipStream_t s, const ProfScope& ps) {
  switch (a.mode) {
    case CONV_STORE: conv_dispatch3<KIND, KSPLIT, CONV_STORE>(a, grid, nt, s, ps); break;
    case CONV_ACCUM: conv_dispatch3<KIND, KSPLIT, CONV_ACCUM>(a, grid, nt, s, ps); break;
    case CONV_STORE_T: conv_dispatch3<KIND, KSPLIT, CONV_STORE_T>(a, grid, nt, s, ps); break;
    case CONV_RESID_R: conv_dispatch3<KIND, KSPLIT, CONV_RESID_R>(a, grid, nt, s, ps); break;
    default: conv_dispatch3<KIND, KSPLIT, CONV_RESID_T>(a, grid, nt, s, ps); break;
  }
}

template <int KIND>
void conv_dispatch(const ConvArgs& a, dim3 grid, int nt, bool ksplit, hipStream_t s, const ProfScope& ps) {
  if (ksplit)
    conv_dispatch2<KIND, true>(a, grid, nt, s, ps);
  else
    conv_dispatch2<KIND, false>(a, grid, nt, s, ps);
}

// ---------------------------------------------------------- lift / proj ---
// Per-direction, per-cell diagonal of L in cancellation-free form:
//   d = sum_a |u_a|/h + sT (1 - S_mm) + sA S_mm.
__device__ inline float diag_of(const float* dc, const float* Sd, float st, float sa, int m) {
  const float smm = Sd[m];
  return dc[4 * m + 3] + st * (1.f - smm) + sa * smm;
}

constexpr int PT = 64;  // pixels per block of the lift kernel

// f0[p][c] = sum_m Win[c][m] v[m][p] / d[m][p] for a tile of 64 pixels; when
// t0 is given also t0 = ainv0 (.) f0 (the first smoothing step's input).
// LDS holds v~ as [m][pixel] and W_in transposed as [m][c], so the
// channel-fastest thread order reads consecutive banks.
__global__ __launch_bounds__(256) void lift_kernel(Slots sl, const double* __restrict__ v,
                                                   const double* __restrict__ vs,
                                                   const float* __restrict__ sT, const float* __restrict__ sA,
                                                   const float* __restrict__ dc, const float* __restrict__ Sd,
                                                   const float* __restrict__ Win, float* __restrict__ f0,
                                                   const float* __restrict__ ainv, float* __restrict__ t0, int N,
                                                   int C0, int64_t P, int t16) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  v = at(v, bs.ws + bs.dx);
  const double vsc = vs ? at(vs, bs.ws)[0] : 1.0;
  f0 = at(f0, bs.ws);
  if (t0) {
    t0 = at(t0, bs.ws);
    ainv = at(ainv, bs.op);
  }
  sT = at(sT, bs.op);
  sA = at(sA, bs.op);
  dc = at(dc, bs.op);
  Sd = at(Sd, bs.op);
  extern __shared__ float sm[];
  float* vt = sm;               // [N][PT]
  float* wt = sm + N * PT;      // [N][C0]
  const int64_t p0 = int64_t(blockIdx.x) * PT;
  for (int idx = threadIdx.x; idx < C0 * N; idx += 256) {
    const int c = idx / N, m = idx - c * N;
    wt[m * C0 + c] = Win[idx];
  }
  {
    // loads at a clamped pixel, zeroed afterwards: no branch around them
    const int64_t p = p0 + (threadIdx.x & (PT - 1));
    const int64_t pc = p < P ? p : P - 1;
    const float st = sT[pc], sa = sA[pc];
#pragma unroll 4
    for (int idx = threadIdx.x; idx < N * PT; idx += 256) {
      const int m = idx / PT;
      const float val = float(v[int64_t(m) * P + pc] * vsc) / diag_of(dc, Sd, st, sa, m);
      vt[idx] = p < P ? val : 0.f;
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < PT * C0; idx += 256) {
    const int pl = idx / C0, c = idx - pl * C0;
    const int64_t p = p0 + pl;
    if (p >= P) continue;
    float acc = 0.f;
#pragma unroll 4
    for (int m = 0; m < N; ++m) acc += wt[m * C0 + c] * vt[m * PT + pl];
    const int64_t o = p * C0 + c;
    f0[o] = acc;
    if (t0) {
      if (t16)
        reinterpret_cast<uint16_t*>(t0)[o] = uint16_t(bf16_bits(ainv[o] * acc));
      else
        t0[o] = ainv[o] * acc;
    }
  }
}

// z[m][p] = s v[m][p] / d[m][p] + sum_c Wout[m][c] u0[p][c] for PP pixels
// (64 for up to 64 directions, else 16): thread t owns pixel t % PP and
// directions t / PP + (256 / PP) q; u0 rows are padded in LDS
// (conflict-free) and v is requested before the sum.
template <int DPT, int PP>
__global__ __launch_bounds__(256) void proj_kernel(Slots sl, const double* __restrict__ v,
                                                   const double* __restrict__ vs,
                                                   const float* __restrict__ u0, const float* __restrict__ sT,
                                                   const float* __restrict__ sA, const float* __restrict__ dc,
                                                   const float* __restrict__ Sd, const float* __restrict__ Wout,
                                                   float sc, float* __restrict__ z, int N, int C0, int64_t P) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  v = at(v, bs.ws + bs.dx);
  const double vsc = vs ? at(vs, bs.ws)[0] : 1.0;
  u0 = at(u0, bs.ws);
  z = at(z, bs.ws + bs.dy);
  sT = at(sT, bs.op);
  sA = at(sA, bs.op);
  dc = at(dc, bs.op);
  Sd = at(Sd, bs.op);
  extern __shared__ float sm[];
  const int ld = C0 + 1;
  float* us = sm;              // [PP][C0 + 1]
  float* ws = sm + PP * ld;    // [N][C0]
  const int64_t p0 = int64_t(blockIdx.x) * PP;
  for (int idx = threadIdx.x; idx < PP * C0; idx += 256) {
    const int pl = idx / C0, c = idx - pl * C0;
    const int64_t p = p0 + pl;
    const float u = u0[(p < P ? p : P - 1) * C0 + c];
    us[pl * ld + c] = p < P ? u : 0.f;
  }
#pragma unroll 4
  for (int idx = threadIdx.x; idx < N * C0; idx += 256) ws[idx] = Wout[idx];
  const int pl = threadIdx.x & (PP - 1);
  const int slot = PP == 64 ? __builtin_amdgcn_readfirstlane(int(threadIdx.x) / PP) : int(threadIdx.x) / PP;
  constexpr int NSLOT = 256 / PP;
  const int64_t p = p0 + pl;
  double vv[DPT];
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int m = slot + NSLOT * q;
    const double val = v[int64_t(m < N ? m : N - 1) * P + (p < P ? p : P - 1)];
    vv[q] = (p < P && m < N) ? val : 0.0;
  }
  __syncthreads();
  if (p >= P) return;
  const float st = sT[p], sa = sA[p];
  float acc[DPT];
#pragma unroll
  for (int q = 0; q < DPT; ++q) acc[q] = 0.f;
#pragma unroll 4
  for (int c = 0; c < C0; ++c) {
    const float u = us[pl * ld + c];
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int m = slot + NSLOT * q;
      if (m < N) acc[q] += ws[m * C0 + c] * u;
    }
  }
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int m = slot + NSLOT * q;
    if (m >= N) break;
    const int64_t o = int64_t(m) * P + p;
    z[o] = sc * (float(vv[q] * vsc) / diag_of(dc, Sd, st, sa, m)) + acc[q];
  }
}

// Lift and projection with one direction (or channel) slot per wave: a
// block owns 64 pixels, lane = pixel, wave w = rows w, w + 4, ... of the
// 1x1 weights, which are then wave-uniform and come from scalar loads of
// the slot-packed copies (one LDS read feeds CQ or DPT FMAs).  The lift's
// channels-last output goes through LDS so its stores are coalesced.
// Same sums, in the same order, as lift_kernel / proj_kernel.
template <int CQ, int DPT>
__global__ __launch_bounds__(256) void lift_slot_kernel(Slots sl, const double* __restrict__ v,
                                                        const double* __restrict__ vs,
                                                        const float* __restrict__ sT, const float* __restrict__ sA,
                                                        const float* __restrict__ dc, const float* __restrict__ Sd,
                                                        const float* __restrict__ Wp, float* __restrict__ f0,
                                                        const float* __restrict__ ainv, float* __restrict__ t0, int N,
                                                        int64_t P, int t16) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  v = at(v, bs.ws + bs.dx);
  const double vsc = vs ? at(vs, bs.ws)[0] : 1.0;
  f0 = at(f0, bs.ws);
  if (t0) {
    t0 = at(t0, bs.ws);
    ainv = at(ainv, bs.op);
  }
  sT = at(sT, bs.op);
  sA = at(sA, bs.op);
  dc = at(dc, bs.op);
  Sd = at(Sd, bs.op);
  constexpr int C0 = 4 * CQ;
  extern __shared__ float sm[];  // [N][64] scaled v, then [64][C0 + 1] output
  const int lane = threadIdx.x & 63;
  const int slot = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int64_t p0 = int64_t(blockIdx.x) * 64;
  const int64_t p = p0 + lane;
  const int64_t pc = p < P ? p : P - 1;
  const float st = sT[pc], sa = sA[pc];
  double vo[DPT];
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int m = slot + 4 * q;
    vo[q] = v[int64_t(m < N ? m : N - 1) * P + pc];
  }
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int m = slot + 4 * q;
    if (m < N) sm[m * 64 + lane] = p < P ? float(vo[q] * vsc) / diag_of(dc, Sd, st, sa, m) : 0.f;
  }
  __syncthreads();
  float acc[CQ];
#pragma unroll
  for (int q = 0; q < CQ; ++q) acc[q] = 0.f;
  const float* __restrict__ wp = Wp + slot * N * CQ;
#pragma unroll 2
  for (int m = 0; m < N; ++m) {
    const float xv = sm[m * 64 + lane];
#pragma unroll
    for (int q = 0; q < CQ; ++q) acc[q] += wp[m * CQ + q] * xv;
  }
  __syncthreads();
  constexpr int LD = C0 + 1;
#pragma unroll
  for (int q = 0; q < CQ; ++q) sm[lane * LD + slot + 4 * q] = acc[q];
  __syncthreads();
  float ai[CQ];
#pragma unroll
  for (int k = 0; k < CQ; ++k) {
    const int idx = int(threadIdx.x) + 256 * k;
    const int pl = idx / C0, c = idx - (idx / C0) * C0;
    const int64_t pp = p0 + pl;
    ai[k] = t0 ? ainv[(pp < P ? pp : P - 1) * C0 + c] : 0.f;
  }
#pragma unroll
  for (int k = 0; k < CQ; ++k) {
    const int idx = int(threadIdx.x) + 256 * k;
    const int pl = idx / C0, c = idx - (idx / C0) * C0;
    const int64_t pp = p0 + pl;
    if (pp >= P) continue;
    const float val = sm[pl * LD + c];
    f0[pp * C0 + c] = val;
    if (t0) {
      if (t16)
        reinterpret_cast<uint16_t*>(t0)[pp * C0 + c] = uint16_t(bf16_bits(ai[k] * val));
      else
        t0[pp * C0 + c] = ai[k] * val;
    }
  }
}

template <int DPT, int CQ>
__global__ __launch_bounds__(256) void proj_slot_kernel(Slots sl, const double* __restrict__ v,
                                                        const double* __restrict__ vs,
                                                        const float* __restrict__ u0, const float* __restrict__ sT,
                                                        const float* __restrict__ sA, const float* __restrict__ dc,
                                                        const float* __restrict__ Sd, const float* __restrict__ Wp,
                                                        float sc, float* __restrict__ z, int N, int64_t P) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  v = at(v, bs.ws + bs.dx);
  const double vsc = vs ? at(vs, bs.ws)[0] : 1.0;
  u0 = at(u0, bs.ws);
  z = at(z, bs.ws + bs.dy);
  sT = at(sT, bs.op);
  sA = at(sA, bs.op);
  dc = at(dc, bs.op);
  Sd = at(Sd, bs.op);
  constexpr int C0 = 4 * CQ;
  constexpr int LD = C0 + 1;
  extern __shared__ float us[];  // [64][C0 + 1]
  const int lane = threadIdx.x & 63;
  const int slot = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int64_t p0 = int64_t(blockIdx.x) * 64;
  const int64_t p = p0 + lane;
  const int64_t pc = p < P ? p : P - 1;
  float ut[CQ];
#pragma unroll
  for (int k = 0; k < CQ; ++k) {
    const int idx = int(threadIdx.x) + 256 * k;
    const int pl = idx / C0, c = idx - (idx / C0) * C0;
    const int64_t pp = p0 + pl;
    const float u = u0[(pp < P ? pp : P - 1) * C0 + c];
    ut[k] = pp < P ? u : 0.f;
  }
  double vv[DPT];
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int m = slot + 4 * q;
    vv[q] = v[int64_t(m < N ? m : N - 1) * P + pc];
  }
#pragma unroll
  for (int k = 0; k < CQ; ++k) {
    const int idx = int(threadIdx.x) + 256 * k;
    const int pl = idx / C0, c = idx - (idx / C0) * C0;
    us[pl * LD + c] = ut[k];
  }
  __syncthreads();
  float acc[DPT];
#pragma unroll
  for (int q = 0; q < DPT; ++q) acc[q] = 0.f;
  const float* __restrict__ wp = Wp + slot * C0 * DPT;
#pragma unroll 2
  for (int c = 0; c < C0; ++c) {
    const float u = us[lane * LD + c];
#pragma unroll
    for (int q = 0; q < DPT; ++q) acc[q] += wp[c * DPT + q] * u;
  }
  if (p >= P) return;
  const float st = sT[p], sa = sA[p];
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int m = slot + 4 * q;
    if (m >= N) break;
    z[int64_t(m) * P + p] = sc * (float(vv[q] * vsc) / diag_of(dc, Sd, st, sa, m)) + acc[q];
  }
}

__global__ void scale_fields_kernel(Slots sl, const float* __restrict__ ainv, const float* __restrict__ f,
                                    float* __restrict__ t, int64_t n, int t16) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  ainv = at(ainv, bs.op);
  f = at(f, bs.ws);
  t = at(t, bs.ws);
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (; i < n; i += int64_t(gridDim.x) * blockDim.x) {
    if (t16)
      reinterpret_cast<uint16_t*>(t)[i] = uint16_t(bf16_bits(ainv[i] * f[i]));
    else
      t[i] = ainv[i] * f[i];
  }
}

template <class T>
__global__ void fill_kernel(Slots sl, T* p, T v, int64_t n) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  p = at(p, bs.ws);
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}

__global__ void cast_kernel(Slots sl, const double* __restrict__ a, const double* __restrict__ scale,
                            float* __restrict__ b, int64_t n) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  a = at(a, bs.ws + bs.dx);
  b = at(b, bs.ws + bs.dy);
  const double sc = scale ? at(scale, bs.ws)[0] : 1.0;
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (; i < n; i += int64_t(gridDim.x) * blockDim.x) b[i] = float(a[i] * sc);
}

__global__ void copy64_kernel(Slots sl, const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  a = at(a, bs.ws);
  b = at(b, bs.ws);
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (; i < n; i += int64_t(gridDim.x) * blockDim.x) b[i] = a[i];
}

unsigned ew_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return unsigned(g);
}

// ------------------------------------------------------------- CoeffNet ---
// Direct 3^d convolution with bias and ReLU, one thread per output value.
// Channel counts are tiny (3 .. coef_ch 2^l); this runs once per operator.
__global__ void coef_conv_kernel(const float* __restrict__ in, int cin, int ix, int iy, int iz,
                                 const float* __restrict__ w, const float* __restrict__ b,
                                 float* __restrict__ out, int cout, int ox, int oy, int oz, int dim,
                                 int stride) {
  const int64_t total = int64_t(ox) * oy * oz * cout;
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int co = int(idx % cout);
  const int64_t p = idx / cout;
  const int X = int(p % ox), Y = int((p / ox) % oy), Z = int(p / (int64_t(ox) * oy));
  const int taps = dim == 3 ? 27 : 9;
  float acc = b[co];
  for (int t = 0; t < taps; ++t) {
    int k[3], off[3];
    conv3_tap(dim, t, k, off);
    const int x = stride * X + off[0], y = stride * Y + off[1], z = stride * Z + off[2];
    if (x < 0 || x >= ix || y < 0 || y >= iy || z < 0 || z >= iz) continue;
    const float* src = in + ((int64_t(z) * iy + y) * ix + x) * cin;
    const float* wt = w + size_t(co) * cin * taps + t;
    for (int ci = 0; ci < cin; ++ci) acc += wt[size_t(ci) * taps] * src[ci];
  }
  out[idx] = acc > 0.f ? acc : 0.f;
}

__global__ void head_kernel(const float* __restrict__ F, int c, const float* __restrict__ w,
                            const float* __restrict__ b, float* __restrict__ out, int C, int64_t P) {
  int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= P * C) return;
  const int co = int(idx % C);
  const int64_t p = idx / C;
  float acc = b[co];
  for (int ci = 0; ci < c; ++ci) acc += w[size_t(co) * c + ci] * F[p * c + ci];
  out[idx] = acc;
}

}  // namespace

// ------------------------------------------------------------ launchers ---
void conv3_setup(ConvLaunch& c, int dim, const int in_dim[3], int stride) {
  c.dim = dim;
  c.cstride = stride;
  c.ostride = 1;
  c.nclass = 1;
  c.ntap = dim == 3 ? 27 : 9;
  for (int a = 0; a < 3; ++a) {
    c.in_dim[a] = in_dim[a];
    c.g_dim[a] = (a < dim && stride == 2) ? in_dim[a] / 2 : in_dim[a];
    c.out_dim[a] = c.g_dim[a];
    c.obase[0][a] = 0;
  }
  for (int t = 0; t < c.ntap; ++t) {
    int k[3], off[3];
    conv3_tap(dim, t, k, off);
    for (int a = 0; a < 3; ++a) c.toff[t][a] = int8_t(off[a]);
  }
}

void convT4_setup(ConvLaunch& c, int dim, const int in_dim[3]) {
  c.dim = dim;
  c.cstride = 1;
  c.ostride = 2;
  c.nclass = 1 << dim;
  c.ntap = 1 << dim;
  for (int a = 0; a < 3; ++a) {
    c.in_dim[a] = in_dim[a];
    c.g_dim[a] = in_dim[a];
    c.out_dim[a] = a < dim ? 2 * in_dim[a] : in_dim[a];
  }
  for (int cls = 0; cls < c.nclass; ++cls) {
    for (int a = 0; a < 3; ++a) c.obase[cls][a] = int8_t(a < dim ? (cls >> a) & 1 : 0);
    for (int t = 0; t < c.ntap; ++t) {
      int k[3], off[3];
      convT4_tap(dim, cls, t, k, off);
      for (int a = 0; a < 3; ++a) c.toff[cls * c.ntap + t][a] = int8_t(off[a]);
    }
  }
}

void launch_conv(const ConvLaunch& c, int kind, hipStream_t s) {
  RTE_REQUIRE(c.cin % 16 == 0 && c.cout % 16 == 0, RTE_EINVAL, "conv channels must be multiples of 16");
  RTE_REQUIRE(c.nclass * c.ntap <= 64 && c.nclass <= 8, RTE_EINVAL, "conv tap table overflow");
  ConvArgs a;
  a.sl = c.sl;
  a.in = c.in;
  a.out = c.out;
  a.out2 = c.out2;
  a.f = c.f;
  a.a = c.a;
  a.ainv = c.ainv;
  for (int i = 0; i < 3; ++i) {
    a.in_dim[i] = c.in_dim[i];
    a.out_dim[i] = c.out_dim[i];
    a.g_dim[i] = c.g_dim[i];
  }
  a.cin = c.cin;
  a.cout = c.cout;
  a.cstride = c.cstride;
  a.ostride = c.ostride;
  a.ntap = c.ntap;
  a.mode = c.mode;
  a.transposed = c.ostride == 2 ? 1 : 0;
  a.dim = c.dim;
  RTE_REQUIRE(c.w->taps == c.nclass * c.ntap && c.w->cin == c.cin && c.w->cout == c.cout, RTE_EINVAL,
              "conv weights do not match the launch");
  // the residual epilogues read the input at the output pixel
  if (c.mode == CONV_RESID_R || c.mode == CONV_RESID_T)
    RTE_REQUIRE(c.cin == c.cout && c.cstride == 1 && c.ostride == 1, RTE_EINVAL, "bad residual conv");
  if (c.mode == CONV_STORE_T) RTE_REQUIRE(c.out2 && c.ainv, RTE_EINVAL, "dual store needs out2 and ainv");
  const int64_t gm = int64_t(c.g_dim[0]) * c.g_dim[1] * c.g_dim[2];
  const int64_t row_units = (gm + 15) / 16;
  // Tile choice: the widest output-channel tile that still yields >= 2048
  // waves; otherwise 16x16 tiles with the reduction split over the 4 waves
  // of a block (when there are enough k-steps to share).
  const int kc = (kind == MFMA_F32 || c.cin % 32 != 0) ? 16 : 32;
  const int nks = c.ntap * (c.cin / kc);
  const int64_t target = 2048;
  int nt = 0;
  for (int cand : {4, 2, 1})
    if (c.cout % (16 * cand) == 0 && row_units * (c.cout / (16 * cand)) * c.nclass >= target) {
      nt = cand;
      break;
    }
  bool ksplit = false;
  if (nt == 0) {
    nt = 1;
    ksplit = nks >= 8;
  }
  dim3 grid(unsigned(ksplit ? row_units : (row_units + 3) / 4), unsigned(c.cout / (nt * 16)),
            unsigned(c.nclass * c.sl.count));
  // The LDS-staged kernel covers 3x3 stride-1 2D convolutions with BF16
  // weights on grids whose width is a multiple of 16 (64-pixel blocks must
  // tile the grid: segments of one row, or whole rows of a narrow grid).
  const int gxv = c.g_dim[0], gyv = c.g_dim[1];
  const bool lds_ok = kind == MFMA_BF16 && c.dim == 2 && c.ostride == 1 && c.cstride == 1 && c.ntap == 9 &&
                      c.cin % 32 == 0 && gxv % 16 == 0 &&
                      (ksplit ? true : (gxv >= 64 ? gxv % 64 == 0 : (64 % gxv == 0 && gyv % (64 / gxv) == 0)));
  ProfScope ps(RTE_K_CONV, s, true);
  ps.work = 2.0 * double(gm) * c.cout * double(c.cin) * c.ntap * c.nclass;
  ps.key = 0;
  while ((2 << ps.key) <= c.cout && ps.key + 1 < RTE_PROF_KEYS) ++ps.key;  // floor(log2(cout))
  {
    // algorithmic bytes: input tensor, weights, output and epilogue tensors once
    const double in_el = double(c.in_dim[0]) * c.in_dim[1] * c.in_dim[2] * c.cin;
    const double out_el = double(gm) * c.nclass * c.cout;
    const double wbytes = double(c.w->taps) * c.cout * c.cin * (kind == MFMA_F32 ? 4.0 : 2.0);
    const double extra[] = {0.0, 1.0, 2.0, 2.0, 3.0};  // STORE, ACCUM, STORE_T, RESID_R, RESID_T
    ps.bytes = (c.in16 ? 2.0 : 4.0) * in_el + wbytes + 4.0 * out_el * (1.0 + extra[c.mode]);
    if (c.t16) ps.bytes -= 2.0 * out_el;  // the t output (out, or out2 of STORE_T) in 2 bytes
  }
  // The tiled kernel covers every 2D BF16 convolution whose channel counts
  // are multiples of 32 and whose virtual grid is a multiple of 8 per axis.
  int ck = -1;
  if (kind == MFMA_BF16 && c.dim == 2 && c.cin % 32 == 0 && c.cout % 32 == 0 && gxv % 8 == 0 && gyv % 8 == 0) {
    if (c.ostride == 1 && c.cstride == 1 && c.ntap == 9) ck = 0;
    else if (c.ostride == 1 && c.cstride == 2 && c.ntap == 9) ck = 1;
    else if (c.ostride == 2 && c.nclass == 4 && c.ntap == 4) ck = 2;
  }
  // The 3D tiled kernel: 3x3x3 stride-1 and 4x4x4 transposed BF16
  // convolutions, channel counts multiples of 16 (launch_conv requires
  // that), virtual grid a multiple of 4 per axis.
  int ck3 = -1;
  if (kind == MFMA_BF16 && c.dim == 3 && gxv % 4 == 0 && gyv % 4 == 0 && c.g_dim[2] % 4 == 0) {
    if (c.ostride == 1 && c.cstride == 1 && c.ntap == 27) ck3 = 0;
    else if (c.ostride == 2 && c.nclass == 8 && c.ntap == 8) ck3 = 2;
  }
  // BF16-stored t tensors exist only in the tiled 2D kernel's stride-1 and
  // restriction forms
  RTE_REQUIRE(!(c.in16 || c.t16) || ck == 0 || ck == 1, RTE_EINVAL, "conv: BF16 t storage needs the tiled kernel");
  RTE_REQUIRE(!c.in16 || c.mode == CONV_STORE || c.mode == CONV_ACCUM || c.mode == CONV_STORE_T, RTE_EINVAL,
              "conv: a BF16 input is a t tensor");
  RTE_REQUIRE(!c.t16 || c.mode == CONV_RESID_T || c.mode == CONV_RESID_R || c.mode == CONV_STORE_T, RTE_EINVAL,
              "conv: only t outputs are stored as BF16");
  if (ck3 >= 0) {
    a.w = c.w->d16;
    const int nz = c.nclass * c.sl.count;
    if (ck3 == 0) tile3_dispatch<0>(a, nz, c.mode, s, ps);
    else tile3_dispatch<2>(a, nz, c.mode, s, ps);
  } else if (ck >= 0) {
    a.w = c.w->d16;
    const int nz = c.nclass * c.sl.count;
    if (ck == 0) tile_dispatch<0>(a, gxv, gyv, nz, c.mode, c.in16 != 0, c.t16 != 0, s, ps);
    else if (ck == 1) tile_dispatch<1>(a, gxv, gyv, nz, c.mode, c.in16 != 0, c.t16 != 0, s, ps);
    else tile_dispatch<2>(a, gxv, gyv, nz, c.mode, false, false, s, ps);
  } else if (lds_ok) {
    const int rows = ksplit ? 16 : 64;
    const int width = gxv >= rows ? rows : gxv;
    const int nrow = gxv >= rows ? 1 : rows / gxv;
    size_t lds = size_t(2) * (width + 2) * (nrow + 2) * LDS_PIX_WORDS * 4;
    if (ksplit) lds = std::max(lds, size_t(3) * nt * 4 * 64 * 4);
    a.w = c.w->d16;
    const dim3 g2(unsigned((gm + rows - 1) / rows), grid.y, unsigned(c.sl.count));
    if (ksplit)
      lds_dispatch2<true>(a, g2, nt, lds, s, ps);
    else
      lds_dispatch2<false>(a, g2, nt, lds, s, ps);
  } else if (kind == MFMA_F32) {
    a.w = c.w->d32;
    conv_dispatch<0>(a, grid, nt, ksplit, s, ps);
  } else if (c.cin % 32 == 0) {
    a.w = c.w->d16;
    conv_dispatch<2>(a, grid, nt, ksplit, s, ps);
  } else {
    a.w = c.w->d16;
    conv_dispatch<1>(a, grid, nt, ksplit, s, ps);
  }
  RTE_HIP(hipGetLastError());
}

namespace {
// Dispatch of the slot-per-wave lift / projection; false when the shape has
// no instantiation (the 16-pixel kernels run instead).
template <int DPT>
bool lift_slot_go(const Target& T, const Model& m, const double* v, const double* vs, float* f0,
                  const float* ainv, float* t0, bool t16, hipStream_t s) {
  const Operator& op = *T.op;
  const dim3 grid(unsigned((op.cells + 63) / 64), 1, unsigned(T.sl.count));
  const size_t lds = std::max(size_t(op.ndir) * 64, size_t(64) * (m.c0 + 1)) * sizeof(float);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, T.sl, v, vs, T.arr.sT32, T.arr.sA32, T.arr.dc32,
                       T.arr.Sdiag32, m.d_w_in_p, f0, ainv, t0, op.ndir, op.cells, t16 ? 1 : 0);
  };
  switch (m.c0 / 4) {
    case 4: go(lift_slot_kernel<4, DPT>); return true;
    case 8: go(lift_slot_kernel<8, DPT>); return true;
    case 12: go(lift_slot_kernel<12, DPT>); return true;
    case 16: go(lift_slot_kernel<16, DPT>); return true;
    case 32: go(lift_slot_kernel<32, DPT>); return true;
    default: return false;
  }
}
template <int DPT>
bool proj_slot_go(const Target& T, const Model& m, const double* v, const double* vs, const float* u0, float* z,
                  hipStream_t s) {
  const Operator& op = *T.op;
  const dim3 grid(unsigned((op.cells + 63) / 64), 1, unsigned(T.sl.count));
  const size_t lds = size_t(64) * (m.c0 + 1) * sizeof(float);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, T.sl, v, vs, u0, T.arr.sT32, T.arr.sA32, T.arr.dc32,
                       T.arr.Sdiag32, m.d_w_out_p, m.s, z, op.ndir, op.cells);
  };
  switch (m.c0 / 4) {
    case 4: go(proj_slot_kernel<DPT, 4>); return true;
    case 8: go(proj_slot_kernel<DPT, 8>); return true;
    case 12: go(proj_slot_kernel<DPT, 12>); return true;
    case 16: go(proj_slot_kernel<DPT, 16>); return true;
    case 32: go(proj_slot_kernel<DPT, 32>); return true;
    default: return false;
  }
}
template <class F>
bool by_budget(int N, F&& f) {
  switch (slot_budget(N)) {
    case 1: return f(std::integral_constant<int, 1>());
    case 2: return f(std::integral_constant<int, 2>());
    case 4: return f(std::integral_constant<int, 4>());
    case 8: return f(std::integral_constant<int, 8>());
    case 16: return f(std::integral_constant<int, 16>());
    case 24: return f(std::integral_constant<int, 24>());
    case 32: return f(std::integral_constant<int, 32>());
    default: return false;
  }
}
}  // namespace

void launch_lift(const Target& T, const Model& m, const double* v, const double* vs, float* f0,
                 const float* ainv, float* t0, bool t16, hipStream_t s) {
  const Operator& op = *T.op;
  if (m.d_w_in_p && by_budget(op.ndir, [&](auto b) {
        return lift_slot_go<decltype(b)::value>(T, m, v, vs, f0, ainv, t0, t16, s);
      })) {
    RTE_HIP(hipGetLastError());
    return;
  }
  const size_t lds = (size_t(op.ndir) * PT + size_t(m.c0) * op.ndir) * sizeof(float);
  RTE_REQUIRE(lds <= 64 * 1024, RTE_EINVAL, "lift tile does not fit in LDS");
  const dim3 grid(unsigned((op.cells + PT - 1) / PT), 1, unsigned(T.sl.count));
  hipLaunchKernelGGL(lift_kernel, grid, dim3(256), lds, s, T.sl, v, vs, T.arr.sT32, T.arr.sA32, T.arr.dc32,
                     T.arr.Sdiag32, m.d_w_in, f0, ainv, t0, op.ndir, m.c0, op.cells, t16 ? 1 : 0);
  RTE_HIP(hipGetLastError());
}

void launch_proj(const Target& T, const Model& m, const double* v, const double* vs, const float* u0,
                 float* z, hipStream_t s) {
  const Operator& op = *T.op;
  if (m.d_w_out_p &&
      by_budget(op.ndir, [&](auto b) { return proj_slot_go<decltype(b)::value>(T, m, v, vs, u0, z, s); })) {
    RTE_HIP(hipGetLastError());
    return;
  }
  const bool wide = op.ndir <= 64;
  const int pp = wide ? 64 : 16;
  const size_t lds = (size_t(pp) * (m.c0 + 1) + size_t(op.ndir) * m.c0) * sizeof(float);
  RTE_REQUIRE(lds <= 64 * 1024, RTE_EINVAL, "projection tile does not fit in LDS");
  RTE_REQUIRE(op.ndir <= 256, RTE_EINVAL, "too many directions for the projection");
  const dim3 grid(unsigned((op.cells + pp - 1) / pp), 1, unsigned(T.sl.count));
  const int dpt = (op.ndir + 256 / pp - 1) / (256 / pp);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, T.sl, v, vs, u0, T.arr.sT32, T.arr.sA32, T.arr.dc32,
                       T.arr.Sdiag32, m.d_w_out, m.s, z, op.ndir, m.c0, op.cells);
  };
  if (wide) {
    if (dpt <= 1) go(proj_kernel<1, 64>);
    else if (dpt <= 2) go(proj_kernel<2, 64>);
    else if (dpt <= 4) go(proj_kernel<4, 64>);
    else if (dpt <= 8) go(proj_kernel<8, 64>);
    else go(proj_kernel<16, 64>);
  } else {
    if (dpt <= 8) go(proj_kernel<8, 16>);
    else go(proj_kernel<16, 16>);
  }
  RTE_HIP(hipGetLastError());
}

namespace {
dim3 ew_grid3(int64_t n, const Slots& sl) { return dim3(ew_grid(n), 1, unsigned(sl.count)); }
}  // namespace

void launch_scale_fields(const Slots& sl, const float* ainv, const float* f, float* t, int64_t count, bool t16,
                         hipStream_t s) {
  hipLaunchKernelGGL(scale_fields_kernel, ew_grid3(count, sl), dim3(256), 0, s, sl, ainv, f, t, count,
                     t16 ? 1 : 0);
  RTE_HIP(hipGetLastError());
}

void launch_fill_f32(const Slots& sl, float* p, float v, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel<float>, ew_grid3(count, sl), dim3(256), 0, s, sl, p, v, count);
  RTE_HIP(hipGetLastError());
}

void launch_fill_f64(const Slots& sl, double* p, double v, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel<double>, ew_grid3(count, sl), dim3(256), 0, s, sl, p, v, count);
  RTE_HIP(hipGetLastError());
}

void launch_cast_f64_f32(const Slots& sl, const double* src, const double* scale, float* dst, int64_t count,
                         hipStream_t s) {
  hipLaunchKernelGGL(cast_kernel, ew_grid3(count, sl), dim3(256), 0, s, sl, src, scale, dst, count);
  RTE_HIP(hipGetLastError());
}

void launch_copy_f64(const Slots& sl, const double* src, double* dst, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(copy64_kernel, ew_grid3(count, sl), dim3(256), 0, s, sl, src, dst, count);
  RTE_HIP(hipGetLastError());
}

void launch_coef_conv(const float* in, int cin, const int in_dim[3], const float* w, const float* b,
                      float* out, int cout, const int out_dim[3], int dim, int stride, hipStream_t s) {
  const int64_t total = int64_t(out_dim[0]) * out_dim[1] * out_dim[2] * cout;
  hipLaunchKernelGGL(coef_conv_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, in, cin,
                     in_dim[0], in_dim[1], in_dim[2], w, b, out, cout, out_dim[0], out_dim[1], out_dim[2],
                     dim, stride);
  RTE_HIP(hipGetLastError());
}

void launch_head(const float* F, int c, const float* w, const float* b, float* out, int C, int64_t P,
                 hipStream_t s) {
  const int64_t total = P * C;
  hipLaunchKernelGGL(head_kernel, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, F, c, w, b, out, C, P);
  RTE_HIP(hipGetLastError());
}

}  // namespace rte

// MgNet / CoeffNet kernels (paper Sec. 3.2-3.3).
//
// Activations are channels-last FP32: [pixels][C], pixels ordered x fastest.
// Every convolution is an implicit GEMM: rows are the pixels of a "virtual
// grid" (the output grid, or one parity class of it for the transposed
// convolution), columns are output channels, and the reduction runs over
// taps x input channels.  A 256-thread block computes 64 rows x (16 NT)
// columns; each wave owns 16 rows.  Operands are read straight from global
// memory into MFMA fragments -- each lane loads 4 (or 8) consecutive
// channels of one pixel (16/32 bytes) and the matching 4 (8) input channels
// of one output channel's weights, which are pre-packed [tap][cout][cin] --
// so the reuse of a pixel's channels across output-channel tiles happens in
// registers and the reuse across taps in the caches.
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
#include <cstring>

#include "common.h"
#include "taps.h"

namespace rte {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

struct ConvArgs {
  const float* in;
  const void* w;
  float* out;
  const float* f;
  const float* a;
  const float* ainv;
  int in_dim[3];
  int out_dim[3];
  int g_dim[3];
  int cin, cout, cstride, ostride, ntap, mode;
  int8_t obase[8][3];
  int8_t toff[64][3];
};

__device__ inline short bf16_bits(float v) {
  __bf16 h = __bf16(v);
  return __builtin_bit_cast(short, h);
}

template <int KIND, int NT>
__global__ __launch_bounds__(256) void conv_kernel(const ConvArgs A) {
  constexpr int KPL = KIND == 2 ? 8 : 4;  // channels per lane per k-step
  constexpr int KC = 4 * KPL;             // channels per k-step
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int grp = lane >> 4, li = lane & 15;
  const int cls = blockIdx.z;
  const int gx = A.g_dim[0], gy = A.g_dim[1];
  const int64_t gm = int64_t(gx) * gy * A.g_dim[2];
  const int64_t rbase = int64_t(blockIdx.x) * 64 + wave * 16;
  const int co0 = blockIdx.y * (NT * 16);
  const int64_t row = rbase + li;
  const bool rv = row < gm;
  int X = 0, Y = 0, Z = 0;
  if (rv) {
    X = int(row % gx);
    const int64_t t = row / gx;
    Y = int(t % gy);
    Z = int(t / gy);
  }
  v4f acc[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) acc[nt] = v4f{0.f, 0.f, 0.f, 0.f};

  const int cin = A.cin;
  for (int t = 0; t < A.ntap; ++t) {
    const int tap = cls * A.ntap + t;
    const int ix = A.cstride * X + A.toff[tap][0];
    const int iy = A.cstride * Y + A.toff[tap][1];
    const int iz = A.cstride * Z + A.toff[tap][2];
    const bool inb = rv && ix >= 0 && ix < A.in_dim[0] && iy >= 0 && iy < A.in_dim[1] && iz >= 0 &&
                     iz < A.in_dim[2];
    const int64_t ipix = inb ? (int64_t(iz) * A.in_dim[1] + iy) * A.in_dim[0] + ix : 0;
    const float* ap = A.in + ipix * cin + grp * KPL;
    const size_t wrow = (size_t(tap) * A.cout + co0 + li) * cin + grp * KPL;
    for (int ci0 = 0; ci0 < cin; ci0 += KC) {
      float4 a0 = make_float4(0.f, 0.f, 0.f, 0.f), a1 = a0;
      if (inb) {
        a0 = *reinterpret_cast<const float4*>(ap + ci0);
        if (KPL == 8) a1 = *reinterpret_cast<const float4*>(ap + ci0 + 4);
      }
      if constexpr (KIND == 0) {
        const float* W = static_cast<const float*>(A.w) + wrow + ci0;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const float4 bv = *reinterpret_cast<const float4*>(W + size_t(nt) * 16 * cin);
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.x, bv.x, acc[nt], 0, 0, 0);
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.y, bv.y, acc[nt], 0, 0, 0);
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.z, bv.z, acc[nt], 0, 0, 0);
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.w, bv.w, acc[nt], 0, 0, 0);
        }
      } else if constexpr (KIND == 1) {
        const uint16_t* W = static_cast<const uint16_t*>(A.w) + wrow + ci0;
        const v4s av = v4s{bf16_bits(a0.x), bf16_bits(a0.y), bf16_bits(a0.z), bf16_bits(a0.w)};
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const v4s bv = *reinterpret_cast<const v4s*>(W + size_t(nt) * 16 * cin);
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[nt], 0, 0, 0);
        }
      } else {
        const uint16_t* W = static_cast<const uint16_t*>(A.w) + wrow + ci0;
        v8bf av;
        av[0] = __bf16(a0.x); av[1] = __bf16(a0.y); av[2] = __bf16(a0.z); av[3] = __bf16(a0.w);
        av[4] = __bf16(a1.x); av[5] = __bf16(a1.y); av[6] = __bf16(a1.z); av[7] = __bf16(a1.w);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const v8bf bv = *reinterpret_cast<const v8bf*>(W + size_t(nt) * 16 * cin);
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[nt], 0, 0, 0);
        }
      }
    }
  }

  const int cout = A.cout;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t r = rbase + grp * 4 + j;
    if (r >= gm) continue;
    const int Xo = int(r % gx);
    const int64_t t2 = r / gx;
    const int Yo = int(t2 % gy), Zo = int(t2 / gy);
    const int ox = A.ostride * Xo + A.obase[cls][0];
    const int oy = A.ostride * Yo + A.obase[cls][1];
    const int oz = A.ostride * Zo + A.obase[cls][2];
    const int64_t opix = (int64_t(oz) * A.out_dim[1] + oy) * A.out_dim[0] + ox;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int col = co0 + nt * 16 + li;
      const int64_t o = opix * cout + col;
      const float v = acc[nt][j];
      switch (A.mode) {
        case CONV_STORE: A.out[o] = v; break;
        case CONV_ACCUM: A.out[o] += v; break;
        case CONV_RESID_R: A.out[o] = A.f[o] - v - A.a[o] * A.in[o]; break;
        default: A.out[o] = A.ainv[o] * (A.f[o] - v - A.a[o] * A.in[o]); break;
      }
    }
  }
}

template <int KIND>
void conv_dispatch(const ConvArgs& a, dim3 grid, int nt, hipStream_t s) {
  switch (nt) {
    case 4: hipLaunchKernelGGL((conv_kernel<KIND, 4>), grid, dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((conv_kernel<KIND, 2>), grid, dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((conv_kernel<KIND, 1>), grid, dim3(256), 0, s, a); break;
  }
}

// ---------------------------------------------------------- lift / proj ---
// Per-direction, per-cell diagonal of L in cancellation-free form:
//   d = sum_a |u_a|/h + sT (1 - S_mm) + sA S_mm.
__device__ inline float diag_of(const float* dc, const float* Sd, float st, float sa, int m) {
  const float smm = Sd[m];
  return dc[4 * m + 3] + st * (1.f - smm) + sa * smm;
}

// f0[p][c] = sum_m Win[c][m] v[m][p] / d[m][p] for a tile of 64 pixels.
__global__ __launch_bounds__(256) void lift_kernel(const double* __restrict__ v, const float* __restrict__ sT,
                                                   const float* __restrict__ sA, const float* __restrict__ dc,
                                                   const float* __restrict__ Sd, const float* __restrict__ Win,
                                                   float* __restrict__ f0, int N, int C0, int64_t P) {
  extern __shared__ float sm[];
  float* vt = sm;               // [N][64]
  float* w = sm + N * 64;       // [C0][N]
  const int64_t p0 = int64_t(blockIdx.x) * 64;
  for (int idx = threadIdx.x; idx < C0 * N; idx += 256) w[idx] = Win[idx];
  for (int idx = threadIdx.x; idx < N * 64; idx += 256) {
    const int m = idx >> 6;
    const int64_t p = p0 + (idx & 63);
    float val = 0.f;
    if (p < P) val = float(v[int64_t(m) * P + p]) / diag_of(dc, Sd, sT[p], sA[p], m);
    vt[idx] = val;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < 64 * C0; idx += 256) {
    const int pl = idx / C0, c = idx - pl * C0;
    const int64_t p = p0 + pl;
    if (p >= P) continue;
    float acc = 0.f;
    for (int m = 0; m < N; ++m) acc += w[c * N + m] * vt[m * 64 + pl];
    f0[p * C0 + c] = acc;
  }
}

// z[m][p] = s v[m][p] / d[m][p] + sum_c Wout[m][c] u0[p][c].
__global__ __launch_bounds__(256) void proj_kernel(const double* __restrict__ v, const float* __restrict__ u0,
                                                   const float* __restrict__ sT, const float* __restrict__ sA,
                                                   const float* __restrict__ dc, const float* __restrict__ Sd,
                                                   const float* __restrict__ Wout, float sc, float* __restrict__ z,
                                                   int N, int C0, int64_t P) {
  extern __shared__ float sm[];
  const int ld = C0 + 1;
  float* us = sm;  // [64][C0 + 1]
  const int64_t p0 = int64_t(blockIdx.x) * 64;
  for (int idx = threadIdx.x; idx < 64 * C0; idx += 256) {
    const int pl = idx / C0, c = idx - pl * C0;
    const int64_t p = p0 + pl;
    us[pl * ld + c] = p < P ? u0[p * C0 + c] : 0.f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int64_t p = p0 + lane;
  if (p >= P) return;
  const float st = sT[p], sa = sA[p];
  for (int m = wave; m < N; m += 4) {
    float acc = 0.f;
    for (int c = 0; c < C0; ++c) acc += Wout[m * C0 + c] * us[lane * ld + c];
    const int64_t o = int64_t(m) * P + p;
    z[o] = sc * (float(v[o]) / diag_of(dc, Sd, st, sa, m)) + acc;
  }
}

__global__ void scale_fields_kernel(const float* __restrict__ ainv, const float* __restrict__ f,
                                    float* __restrict__ t, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (; i < n; i += int64_t(gridDim.x) * blockDim.x) t[i] = ainv[i] * f[i];
}

template <class T>
__global__ void fill_kernel(T* p, T v, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (; i < n; i += int64_t(gridDim.x) * blockDim.x) p[i] = v;
}

__global__ void cast_kernel(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (; i < n; i += int64_t(gridDim.x) * blockDim.x) b[i] = float(a[i]);
}

__global__ void copy64_kernel(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
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
  a.in = c.in;
  a.out = c.out;
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
  std::memset(a.obase, 0, sizeof(a.obase));
  std::memset(a.toff, 0, sizeof(a.toff));
  for (int k = 0; k < c.nclass; ++k)
    for (int i = 0; i < 3; ++i) a.obase[k][i] = c.obase[k][i];
  for (int k = 0; k < c.nclass * c.ntap; ++k)
    for (int i = 0; i < 3; ++i) a.toff[k][i] = c.toff[k][i];
  RTE_REQUIRE(c.w->taps == c.nclass * c.ntap && c.w->cin == c.cin && c.w->cout == c.cout, RTE_EINVAL,
              "conv weights do not match the launch");
  // the residual epilogues read the input at the output pixel
  if (c.mode == CONV_RESID_R || c.mode == CONV_RESID_T)
    RTE_REQUIRE(c.cin == c.cout && c.cstride == 1 && c.ostride == 1, RTE_EINVAL, "bad residual conv");
  const int64_t gm = int64_t(c.g_dim[0]) * c.g_dim[1] * c.g_dim[2];
  const int nt = c.cout % 64 == 0 ? 4 : (c.cout % 32 == 0 ? 2 : 1);
  dim3 grid(unsigned((gm + 63) / 64), unsigned(c.cout / (nt * 16)), unsigned(c.nclass));
  ProfScope ps(RTE_K_CONV, s);
  ps.work = 2.0 * double(gm) * c.cout * double(c.cin) * c.ntap * c.nclass;
  if (kind == MFMA_F32) {
    a.w = c.w->d32;
    conv_dispatch<0>(a, grid, nt, s);
  } else if (c.cin % 32 == 0) {
    a.w = c.w->d16;
    conv_dispatch<2>(a, grid, nt, s);
  } else {
    a.w = c.w->d16;
    conv_dispatch<1>(a, grid, nt, s);
  }
  RTE_HIP(hipGetLastError());
}

void launch_lift(const Operator& op, const Model& m, const double* v, float* f0, hipStream_t s) {
  const size_t lds = (size_t(op.ndir) * 64 + size_t(m.c0) * op.ndir) * sizeof(float);
  RTE_REQUIRE(lds <= 64 * 1024, RTE_EINVAL, "lift tile does not fit in LDS");
  hipLaunchKernelGGL(lift_kernel, dim3(unsigned((op.cells + 63) / 64)), dim3(256), lds, s, v, op.sT32, op.sA32,
                     op.dc32, op.Sdiag32, m.d_w_in, f0, op.ndir, m.c0, op.cells);
  RTE_HIP(hipGetLastError());
}

void launch_proj(const Operator& op, const Model& m, const double* v, const float* u0, float* z,
                 hipStream_t s) {
  const size_t lds = size_t(64) * (m.c0 + 1) * sizeof(float);
  RTE_REQUIRE(lds <= 64 * 1024, RTE_EINVAL, "projection tile does not fit in LDS");
  hipLaunchKernelGGL(proj_kernel, dim3(unsigned((op.cells + 63) / 64)), dim3(256), lds, s, v, u0, op.sT32,
                     op.sA32, op.dc32, op.Sdiag32, m.d_w_out, m.s, z, op.ndir, m.c0, op.cells);
  RTE_HIP(hipGetLastError());
}

void launch_scale_fields(const float* ainv, const float* f, float* t, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(scale_fields_kernel, dim3(ew_grid(count)), dim3(256), 0, s, ainv, f, t, count);
  RTE_HIP(hipGetLastError());
}

void launch_fill_f32(float* p, float v, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel<float>, dim3(ew_grid(count)), dim3(256), 0, s, p, v, count);
  RTE_HIP(hipGetLastError());
}

void launch_fill_f64(double* p, double v, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(fill_kernel<double>, dim3(ew_grid(count)), dim3(256), 0, s, p, v, count);
  RTE_HIP(hipGetLastError());
}

void launch_cast_f64_f32(const double* src, float* dst, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(cast_kernel, dim3(ew_grid(count)), dim3(256), 0, s, src, dst, count);
  RTE_HIP(hipGetLastError());
}

void launch_copy_f64(const double* src, double* dst, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(copy64_kernel, dim3(ew_grid(count)), dim3(256), 0, s, src, dst, count);
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

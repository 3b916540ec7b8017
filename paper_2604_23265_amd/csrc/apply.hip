// Discrete-ordinates operator apply (eq. (DORTE_2d), step-upwind finite
// volumes): y = L x or y = b - L x, fused streaming + collision + scatter.
//
// Layout: x, y direction-major [N][cells].  A 256-thread block owns 64
// consecutive cells and all N directions.  The block stages x[:, tile] in
// LDS (coalesced rows of 64 cells per direction); each wave then takes four
// directions at a time, one cell per lane: the scatter sum_n S_mn x_n reads
// S through wave-uniform (scalar) loads and x_n from LDS, reusing each LDS
// read for four directions; the upwind neighbour comes from global memory
// (the same or an adjacent row, cached).  Collision uses the
// cancellation-free form sT (x - Sx) + sA Sx = sT x - sS Sx.
#include "common.h"

namespace rte {
namespace {

constexpr int TILE = 64;
constexpr int MB = 4;  // directions per lane per pass

template <class T, class TI, class TO, bool RES, bool LDS>
__global__ __launch_bounds__(256) void apply_kernel(const TI* __restrict__ x, TO* __restrict__ y,
                                                    const double* __restrict__ b,
                                                    const T* __restrict__ sT, const T* __restrict__ sA,
                                                    const T* __restrict__ S, const T* __restrict__ dc,
                                                    const int* __restrict__ sg, int N, int nx, int ny,
                                                    int nz, int64_t cells) {
  extern __shared__ char smem[];
  T* xs = reinterpret_cast<T*>(smem);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int64_t c0 = int64_t(blockIdx.x) * TILE;
  if (LDS) {
    for (int idx = threadIdx.x; idx < N * TILE; idx += 256) {
      int m = idx / TILE, cl = idx - m * TILE;
      int64_t cc = c0 + cl;
      xs[idx] = cc < cells ? T(x[int64_t(m) * cells + cc]) : T(0);
    }
    __syncthreads();
  }
  const int64_t c = c0 + lane;
  if (c >= cells) return;
  const int i = int(c % nx);
  const int64_t rr = c / nx;
  const int j = int(rr % ny);
  const int k = int(rr / ny);
  const int pos[3] = {i, j, k};
  const int ext[3] = {nx, ny, nz};
  const int64_t stride[3] = {1, nx, int64_t(nx) * ny};
  const T st = sT[c], sa = sA[c];
  for (int m0 = wave * MB; m0 < N; m0 += 4 * MB) {
    T acc[MB];
#pragma unroll
    for (int q = 0; q < MB; ++q) acc[q] = T(0);
    if (m0 + MB <= N) {
      for (int n = 0; n < N; ++n) {
        T xv = LDS ? xs[n * TILE + lane] : T(x[int64_t(n) * cells + c]);
#pragma unroll
        for (int q = 0; q < MB; ++q) acc[q] += S[(m0 + q) * N + n] * xv;
      }
    } else {
      for (int n = 0; n < N; ++n) {
        T xv = LDS ? xs[n * TILE + lane] : T(x[int64_t(n) * cells + c]);
        for (int q = 0; q < MB; ++q)
          if (m0 + q < N) acc[q] += S[(m0 + q) * N + n] * xv;
      }
    }
#pragma unroll
    for (int q = 0; q < MB; ++q) {
      const int m = m0 + q;
      if (m >= N) break;
      const int64_t o = int64_t(m) * cells + c;
      const T xc = LDS ? xs[m * TILE + lane] : T(x[o]);
      T str = T(0);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int s = sg[4 * m + a];
        if (s == 0) continue;
        const int p = pos[a] - s;
        const T xn = (p >= 0 && p < ext[a]) ? T(x[o - s * stride[a]]) : T(0);
        str += dc[4 * m + a] * (xc - xn);
      }
      const T val = str + st * (xc - acc[q]) + sa * acc[q];
      if (RES)
        y[o] = TO(b[o] - double(val));
      else
        y[o] = TO(val);
    }
  }
}

template <class T, class TI, class TO, bool RES>
void go(const Operator& op, const void* x, void* y, const double* b, hipStream_t s) {
  const T* sT;
  const T* sA;
  const T* S;
  const T* dc;
  if constexpr (sizeof(T) == 8) {
    sT = op.sT64; sA = op.sA64; S = op.S64; dc = op.dc64;
  } else {
    sT = op.sT32; sA = op.sA32; S = op.S32; dc = op.dc32;
  }
  const size_t lds = size_t(op.ndir) * TILE * sizeof(T);
  const unsigned grid = unsigned((op.cells + TILE - 1) / TILE);
  if (lds <= 48 * 1024) {
    hipLaunchKernelGGL((apply_kernel<T, TI, TO, RES, true>), dim3(grid), dim3(256), lds, s,
                       static_cast<const TI*>(x), static_cast<TO*>(y), b, sT, sA, S, dc, op.dsgn,
                       op.ndir, op.nx, op.ny, op.nz, op.cells);
  } else {
    hipLaunchKernelGGL((apply_kernel<T, TI, TO, RES, false>), dim3(grid), dim3(256), 0, s,
                       static_cast<const TI*>(x), static_cast<TO*>(y), b, sT, sA, S, dc, op.dsgn,
                       op.ndir, op.nx, op.ny, op.nz, op.cells);
  }
  RTE_HIP(hipGetLastError());
}

}  // namespace

void launch_apply(const Operator& op, const void* x, int tin, void* y, int tout, const double* b,
                  bool fp64, hipStream_t s) {
  const double unknowns = double(op.n), cells = double(op.cells);
  if (b) {
    RTE_REQUIRE(fp64 && tin == 1 && tout == 1, RTE_EINVAL, "residual is FP64 only");
    ProfScope ps(RTE_K_RESIDUAL, s);
    ps.work = 24.0 * unknowns + 16.0 * cells;  // x, b in; r out; sT, sA
    go<double, double, double, true>(op, x, y, b, s);
    return;
  }
  ProfScope ps(RTE_K_APPLY, s);
  const double esz[2] = {4.0, 8.0};
  ps.work = (esz[tin] + esz[tout]) * unknowns + (fp64 ? 16.0 : 8.0) * cells;
  if (fp64) {
    RTE_REQUIRE(tin == 1 && tout == 1, RTE_EINVAL, "FP64 apply takes FP64 vectors");
    go<double, double, double, false>(op, x, y, nullptr, s);
  } else if (tin == 0 && tout == 0) {
    go<float, float, float, false>(op, x, y, nullptr, s);
  } else if (tin == 0 && tout == 1) {
    go<float, float, double, false>(op, x, y, nullptr, s);
  } else {
    go<float, double, float, false>(op, x, y, nullptr, s);
  }
}

}  // namespace rte

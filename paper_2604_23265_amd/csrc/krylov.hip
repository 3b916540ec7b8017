// FP64 Krylov kernels for flexible GMRES: two-pass classical Gram-Schmidt
// (CGS2), on-device Givens / Hessenberg least squares, and the solution
// update.  Every reduction is two-stage with a fixed assignment of elements
// to blocks and a fixed combination order, so results are bitwise
// reproducible for a given n regardless of what else runs on the device.
//
// Vectors are contiguous FP64 arrays of length n; the basis V is a set of
// vectors spaced ldv apart.  Partial sums go to part[blk * ldp + i].
#include "common.h"

namespace rte {
namespace {

constexpr int KT = 256;      // threads per block
constexpr int NVB = 8;       // basis vectors per pass in the dot kernels
constexpr int HMAX = 65;     // max basis vectors (restart <= 64)

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of one value per thread over the block, in a fixed order; result valid
// in every thread.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0;
#pragma unroll
  for (int i = 0; i < KT / 64; ++i) s += red[i];
  return s;
}

// Block b owns elements [b * chunk, min(n, (b + 1) * chunk)) with
// chunk = ceil(n / nblk); computed in 32 bits (n < 2^31).
__device__ inline void chunk_of(int64_t n, int nblk, int64_t& beg, int64_t& end) {
  const unsigned nn = unsigned(n);
  const unsigned chunk = (nn + unsigned(nblk) - 1u) / unsigned(nblk);
  beg = int64_t(blockIdx.x) * chunk;
  end = beg + chunk < n ? beg + chunk : n;
}

// part[blk][i] = sum over the block's chunk of V_i . w, i < nv.
__device__ __attribute__((always_inline)) inline void dots_body(const double* __restrict__ V, int64_t ldv, int nv,
                                 const double* __restrict__ w, int64_t n, double* __restrict__ part,
                                 int nblk, double* red) {
  int64_t beg, end;
  chunk_of(n, nblk, beg, end);
  for (int vb = 0; vb < nv; vb += NVB) {
    double acc[NVB];
#pragma unroll
    for (int q = 0; q < NVB; ++q) acc[q] = 0.0;
    const int cnt = nv - vb < NVB ? nv - vb : NVB;
#pragma unroll 4
    for (int64_t e = beg + threadIdx.x; e < end; e += KT) {
      const double we = w[e];
#pragma unroll
      for (int q = 0; q < NVB; ++q)
        if (q < cnt) acc[q] += V[int64_t(vb + q) * ldv + e] * we;
    }
#pragma unroll
    for (int q = 0; q < NVB; ++q) {
      if (q >= cnt) break;
      const double s = block_sum(acc[q], red);
      if (threadIdx.x == 0) part[int64_t(blockIdx.x) * HMAX + vb + q] = s;
    }
  }
}

__global__ __launch_bounds__(KT) void dots_kernel(const double* __restrict__ V, int64_t ldv, int nv,
                                                  const double* __restrict__ w, int64_t n,
                                                  double* __restrict__ part, int nblk) {
  __shared__ double red[KT / 64];
  dots_body(V, ldv, nv, w, n, part, nblk, red);
}

// w -= sum_i h_i V_i, then the partial dots of the updated w with every V_i.
__global__ __launch_bounds__(KT) void update_dots_kernel(const double* __restrict__ V, int64_t ldv, int nv,
                                                         const double* __restrict__ h, double* __restrict__ w,
                                                         int64_t n, double* __restrict__ part, int nblk) {
  __shared__ double red[KT / 64];
  __shared__ double hs[HMAX];
  if (threadIdx.x < nv) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  int64_t beg, end;
  chunk_of(n, nblk, beg, end);
  for (int64_t e = beg + threadIdx.x; e < end; e += KT) {
    double acc = w[e];
#pragma unroll 8
    for (int i = 0; i < nv; ++i) acc -= hs[i] * V[int64_t(i) * ldv + e];
    w[e] = acc;
  }
  // the dots re-read this block's own chunk of w, written by its own threads
  __syncthreads();
  dots_body(V, ldv, nv, w, n, part, nblk, red);
}

// w -= sum_i h_i V_i, then the partial sums of w^2.
__global__ __launch_bounds__(KT) void update_norm_kernel(const double* __restrict__ V, int64_t ldv, int nv,
                                                         const double* __restrict__ h, double* __restrict__ w,
                                                         int64_t n, double* __restrict__ part, int nblk) {
  __shared__ double red[KT / 64];
  __shared__ double hs[HMAX];
  if (threadIdx.x < nv) hs[threadIdx.x] = h[threadIdx.x];
  __syncthreads();
  int64_t beg, end;
  chunk_of(n, nblk, beg, end);
  double ss = 0.0;
  for (int64_t e = beg + threadIdx.x; e < end; e += KT) {
    double acc = w[e];
#pragma unroll 8
    for (int i = 0; i < nv; ++i) acc -= hs[i] * V[int64_t(i) * ldv + e];
    w[e] = acc;
    ss += acc * acc;
  }
  const double s = block_sum(ss, red);
  if (threadIdx.x == 0) part[int64_t(blockIdx.x) * HMAX] = s;
}

// out[i] = sum_blk part[blk][i], one block per i, fixed order.
__global__ __launch_bounds__(KT) void reduce_kernel(const double* __restrict__ part, int nblk,
                                                    double* __restrict__ out) {
  __shared__ double red[KT / 64];
  const int i = blockIdx.x;
  double s = 0;
  for (int b = threadIdx.x; b < nblk; b += KT) s += part[int64_t(b) * HMAX + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[i] = s;
}

// Close Arnoldi step j: assemble column j of the Hessenberg matrix
// (h1 + h2 from the two Gram-Schmidt passes, ||w|| below the diagonal),
// rotate it by the previous Givens rotations, form the new rotation, update
// g, and publish stat = {|g_{j+1}|/||b||, flags, ||w||, 1/||w||}.
// flags: 1 = non-finite value, 2 = ||w|| negligible (the Krylov space is
// invariant: the least-squares solution is exact).
__global__ __launch_bounds__(KT) void finish_kernel(const double* __restrict__ h1, const double* __restrict__ h2,
                                                    const double* __restrict__ partn, int nblk, int j, int k,
                                                    double* __restrict__ H, double* __restrict__ cs,
                                                    double* __restrict__ sn, double* __restrict__ g,
                                                    const double* __restrict__ bnorm, double* __restrict__ stat) {
  __shared__ double red[KT / 64];
  double s = 0;
  for (int b = threadIdx.x; b < nblk; b += KT) s += partn[int64_t(b) * HMAX];
  s = block_sum(s, red);
  if (threadIdx.x != 0) return;
  const double hn = sqrt(s);
  double* col = H + int64_t(j) * (k + 1);
  double cmax = 0;
  for (int i = 0; i <= j; ++i) {
    col[i] = h1[i] + h2[i];
    cmax = fmax(cmax, fabs(col[i]));
  }
  col[j + 1] = hn;
  int flags = 0;
  if (!isfinite(hn) || !isfinite(cmax)) flags |= 1;
  if (hn <= 1e-14 * cmax) flags |= 2;
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double rho = hypot(col[j], col[j + 1]);
  double c = 1.0, sv = 0.0;
  if (rho > 0) {
    c = col[j] / rho;
    sv = col[j + 1] / rho;
  } else {
    flags |= 1;
  }
  cs[j] = c;
  sn[j] = sv;
  col[j] = rho;
  col[j + 1] = 0.0;
  g[j + 1] = -sv * g[j];
  g[j] = c * g[j];
  stat[0] = fabs(g[j + 1]) / bnorm[0];
  stat[1] = double(flags);
  stat[2] = hn;
  stat[3] = hn > 0 ? 1.0 / hn : 0.0;
  if (!isfinite(stat[0])) stat[1] = double(flags | 1);
}

// beta = ||r|| from partial sums; g = beta e_1; stat[3] = 1/beta, stat[4] = beta.
__global__ __launch_bounds__(KT) void start_cycle_kernel(const double* __restrict__ partn, int nblk,
                                                         double* __restrict__ g, int k, double* __restrict__ stat) {
  __shared__ double red[KT / 64];
  double s = 0;
  for (int b = threadIdx.x; b < nblk; b += KT) s += partn[int64_t(b) * HMAX];
  s = block_sum(s, red);
  if (g) {
    for (int i = threadIdx.x; i <= k; i += KT) g[i] = 0.0;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double beta = sqrt(s);
  if (g) g[0] = beta;
  stat[3] = beta > 0 ? 1.0 / beta : 0.0;
  stat[4] = beta;
}

__global__ void scale_kernel(double* __restrict__ w, const double* __restrict__ f, int64_t n) {
  const double a = f[0];
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (; i < n; i += int64_t(gridDim.x) * blockDim.x) w[i] *= a;
}

// Back substitution on the rotated (upper-triangular) Hessenberg matrix.
__global__ void lsq_kernel(const double* __restrict__ H, const double* __restrict__ g, int jj, int k,
                           double* __restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = jj - 1; i >= 0; --i) {
    double s = g[i];
    for (int l = i + 1; l < jj; ++l) s -= H[int64_t(l) * (k + 1) + i] * y[l];
    y[i] = s / H[int64_t(i) * (k + 1) + i];
  }
}

// x += sum_i y_i Z_i (Z stored in FP32).
__global__ __launch_bounds__(KT) void xupdate_kernel(double* __restrict__ x, const float* __restrict__ Z,
                                                     int64_t ldz, const double* __restrict__ y, int jj,
                                                     int64_t n) {
  __shared__ double ys[HMAX];
  if (threadIdx.x < jj) ys[threadIdx.x] = y[threadIdx.x];
  __syncthreads();
  int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (; e < n; e += int64_t(gridDim.x) * blockDim.x) {
    double acc = x[e];
    for (int i = 0; i < jj; ++i) acc += ys[i] * double(Z[int64_t(i) * ldz + e]);
    x[e] = acc;
  }
}

unsigned ew_grid(int64_t n) {
  int64_t g = (n + KT - 1) / KT;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return unsigned(g);
}

}  // namespace

// Partial-sum blocks for a length-n reduction: about 1024 elements per block
// (four per thread), at most 2048 blocks; depends on n only.
int krylov_blocks(int64_t n) {
  int64_t b = (n + 1023) / 1024;
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  return int(b);
}

void launch_dots(const double* V, int64_t ldv, int nv, const double* w, int64_t n, double* part, int nblk,
                 hipStream_t s) {
  RTE_REQUIRE(nv >= 1 && nv <= HMAX, RTE_EINVAL, "too many basis vectors");
  ProfScope ps(RTE_K_ORTH, s, true);
  ps.work = 8.0 * double(n) * (nv + 1);
  launch_k(dots_kernel, dim3(nblk), dim3(KT), 0, s, ps, V, ldv, nv, w, n, part, nblk);
  RTE_HIP(hipGetLastError());
}

void launch_reduce(const double* part, int nblk, int nv, double* out, hipStream_t s) {
  ProfScope ps(RTE_K_ORTH, s, true);
  launch_k(reduce_kernel, dim3(nv), dim3(KT), 0, s, ps, part, nblk, out);
  RTE_HIP(hipGetLastError());
}

void launch_update_dots(const double* V, int64_t ldv, int nv, const double* h, double* w, int64_t n,
                        double* part, int nblk, hipStream_t s) {
  ProfScope ps(RTE_K_ORTH, s, true);
  ps.work = 8.0 * double(n) * (nv + 2);  // V once, w read and written once
  launch_k(update_dots_kernel, dim3(nblk), dim3(KT), 0, s, ps, V, ldv, nv, h, w, n, part, nblk);
  RTE_HIP(hipGetLastError());
}

void launch_update_norm(const double* V, int64_t ldv, int nv, const double* h, double* w, int64_t n,
                        double* part, int nblk, hipStream_t s) {
  ProfScope ps(RTE_K_ORTH, s, true);
  ps.work = 8.0 * double(n) * (nv + 2);
  launch_k(update_norm_kernel, dim3(nblk), dim3(KT), 0, s, ps, V, ldv, nv, h, w, n, part, nblk);
  RTE_HIP(hipGetLastError());
}

void launch_finish_step(const double* h1, const double* h2, const double* partn, int nblk, int j, int k,
                        double* H, double* cs, double* sn, double* g, const double* bnorm, double* stat,
                        hipStream_t s) {
  ProfScope ps(RTE_K_ORTH, s, true);
  launch_k(finish_kernel, dim3(1), dim3(KT), 0, s, ps, h1, h2, partn, nblk, j, k, H, cs, sn, g, bnorm,
                     stat);
  RTE_HIP(hipGetLastError());
}

void launch_scale_by(double* w, const double* stat_inv, int64_t n, hipStream_t s) {
  ProfScope ps(RTE_K_ORTH, s, true);
  ps.work = 16.0 * double(n);
  launch_k(scale_kernel, dim3(ew_grid(n)), dim3(KT), 0, s, ps, w, stat_inv, n);
  RTE_HIP(hipGetLastError());
}

void launch_start_cycle(const double* partn, int nblk, double* g, int k, double* stat, hipStream_t s) {
  hipLaunchKernelGGL(start_cycle_kernel, dim3(1), dim3(KT), 0, s, partn, nblk, g, k, stat);
  RTE_HIP(hipGetLastError());
}

void launch_lsq(const double* H, const double* g, int jj, int k, double* y, hipStream_t s) {
  hipLaunchKernelGGL(lsq_kernel, dim3(1), dim3(64), 0, s, H, g, jj, k, y);
  RTE_HIP(hipGetLastError());
}

void launch_xupdate(double* x, const float* Z, int64_t ldz, const double* y, int jj, int64_t n,
                    hipStream_t s) {
  hipLaunchKernelGGL(xupdate_kernel, dim3(ew_grid(n)), dim3(KT), 0, s, x, Z, ldz, y, jj, n);
  RTE_HIP(hipGetLastError());
}

}  // namespace rte

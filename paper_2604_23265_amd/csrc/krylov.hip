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

// The streaming kernels below keep one element of every basis vector in
// registers: NV is a compile-time register budget (4, 8, 16, 32 or 64 >= nv;
// the 4-vector budget of the first steps saves the clamped reloads, worth
// 1.6 % of the 32-solve C2 batch).  The block sums add lane partners along
// the same lane bits whatever NV is, so the budget does not change results.
// Loads of indices past nv re-read vector nv - 1 (a cached line) and are
// masked arithmetically, so no branch separates the loads of an element.
template <int NV>
__device__ inline void load_column(const double* __restrict__ V, int64_t ldv, int nv, int64_t e, double* v) {
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = V[int64_t(i < nv ? i : nv - 1) * ldv + e];
}

// Block sums of acc[0 .. NV-1] (NV a power of two <= 64), the first cnt of
// them written to part[blk][i].  Within a wave a reduce-scatter halves the
// values each lane carries at every butterfly step (lane bit set: keep the
// upper half), so after log2(NV) steps each lane holds one index, named by
// its high lane bits; the remaining steps add the lanes that share an
// index.  About NV shuffles instead of 6 NV.  The four waves' partials then
// meet in LDS and are added in wave order.  The order of every addition is
// fixed, so results are reproducible.
template <int M, int O>
__device__ inline void reduce_scatter(double* acc, int lane, int& idx) {
  if constexpr (O >= 1) {
    if constexpr (M > 1) {
      constexpr int H = M / 2;
      const bool up = (lane & O) != 0;
#pragma unroll
      for (int k = 0; k < H; ++k) {
        const double send = up ? acc[k] : acc[k + H];
        const double keep = up ? acc[k + H] : acc[k];
        acc[k] = keep + __shfl_xor(send, O, 64);
      }
      if (up) idx += H;
      reduce_scatter<H, O / 2>(acc, lane, idx);
    } else {
      acc[0] += __shfl_xor(acc[0], O, 64);
      reduce_scatter<1, O / 2>(acc, lane, idx);
    }
  }
}

template <int NV>
__device__ inline void block_store(double* acc, int cnt, double* __restrict__ part, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int idx = 0;  // index whose wave sum this lane ends up holding
  reduce_scatter<NV, 32>(acc, lane, idx);
  __syncthreads();
  constexpr int LANES_PER = 64 / NV;  // lanes sharing an index; one of them writes
  if ((lane & (LANES_PER - 1)) == 0) red[wave * NV + idx] = acc[0];
  __syncthreads();
  if (int(threadIdx.x) < cnt) {
    const int i = threadIdx.x;
    part[int64_t(blockIdx.x) * HMAX + i] = ((red[i] + red[NV + i]) + red[2 * NV + i]) + red[3 * NV + i];
  }
}

// part[blk][i] = sum over the block's chunk of V_i . w, i < nv.
template <int NV>
__global__ __launch_bounds__(KT) void dots_kernel(Slots sl, const double* __restrict__ V, int64_t ldv, int nv,
                                                  const double* __restrict__ w, int64_t n,
                                                  double* __restrict__ part, int nblk) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  V = at(V, bs.ws);
  w = at(w, bs.ws);
  part = at(part, bs.ws);
  __shared__ double red[4 * NV];
  int64_t beg, end;
  chunk_of(n, nblk, beg, end);
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  for (int64_t e = beg + threadIdx.x; e < end; e += KT) {
    double v[NV];
    load_column<NV>(V, ldv, nv, e, v);
    const double we = w[e];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += v[i] * we;
  }
  block_store<NV>(acc, nv, part, red);
}

// First Gram-Schmidt correction and the second pass's dots in one read of
// V, for the slot's step j (nv = j + 1 basis vectors, w = V[j + 1]):
// w1 = w - sum_i h_i V_i (written back), then part[blk][i] = V_i . w1
// (i < nv) and part[blk][nv] = w1 . w1.  With HOLD the element's column of V
// stays in registers between the two uses; without it (the widest budget,
// which would not fit) the column is loaded again, from cache.  Up to 8
// vectors a thread takes its elements two at a time, both columns requested
// before either is used: the in-place store of w keeps the compiler from
// moving the next element's loads above it (32 C2 solves, pairs up to 16
// vectors against none, alternating runs: 112.7 -> 107.9 us per launch, and
// 120.7 -> 114.5 us for finish_dots; at 16 vectors the pairs' registers cost
// two of five waves per SIMD, so pairing stops at 8).  Each thread still
// adds its elements in their order: results are unchanged.
template <int NV, bool HOLD>
__global__ __launch_bounds__(KT) void updots_kernel(Slots sl, const double* __restrict__ V, int64_t ldv,
                                                    const double* __restrict__ h, int64_t n,
                                                    double* __restrict__ part, int nblk) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  const int nv = bs.jj + 1;
  V = at(V, bs.ws);
  h = at(h, bs.ws);
  part = at(part, bs.ws);
  double* __restrict__ w = const_cast<double*>(V) + int64_t(nv) * ldv;
  __shared__ double red[4 * NV];
  __shared__ double rww[KT / 64];
  __shared__ double hs[NV];
  if (threadIdx.x < NV) hs[threadIdx.x] = int(threadIdx.x) < nv ? h[threadIdx.x] : 0.0;
  __syncthreads();
  int64_t beg, end;
  chunk_of(n, nblk, beg, end);
  double acc[NV];
  double ww = 0.0;
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  if constexpr (HOLD && NV <= 8) {
    // two elements per trip (e, e + KT: the thread's elements in their order),
    // both columns requested before either is used
    for (int64_t e = beg + threadIdx.x; e < end; e += 2 * KT) {
      const int64_t e2 = e + KT < end ? e + KT : e;
      double v0[NV], v1[NV];
      double x0 = w[e], x1 = w[e2];
      load_column<NV>(V, ldv, nv, e, v0);
      load_column<NV>(V, ldv, nv, e2, v1);
#pragma unroll
      for (int i = 0; i < NV; ++i) x0 -= hs[i] * v0[i];
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += v0[i] * x0;
      w[e] = x0;
      ww += x0 * x0;
      if (e + KT < end) {
#pragma unroll
        for (int i = 0; i < NV; ++i) x1 -= hs[i] * v1[i];
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] += v1[i] * x1;
        w[e2] = x1;
        ww += x1 * x1;
      }
    }
  } else
  for (int64_t e = beg + threadIdx.x; e < end; e += KT) {
    double x = w[e];
    if constexpr (HOLD) {
      double v[NV];
      load_column<NV>(V, ldv, nv, e, v);
#pragma unroll
      for (int i = 0; i < NV; ++i) x -= hs[i] * v[i];
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += v[i] * x;
    } else {
#pragma unroll
      for (int i = 0; i < NV; ++i) x -= hs[i] * V[int64_t(i < nv ? i : nv - 1) * ldv + e];
      __asm__ volatile("" ::: "memory");  // compiler fence: reload the column, do not keep it live
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += V[int64_t(i < nv ? i : nv - 1) * ldv + e] * x;
    }
    w[e] = x;
    ww += x * x;
  }
  const double s = block_sum(ww, rww);
  if (threadIdx.x == 0) part[int64_t(blockIdx.x) * HMAX + nv] = s;
  block_store<NV>(acc, nv, part, red);
}

// First pass of the slot's step j of the lagged CGS2: complete the current
// basis vector in place, V[j] <- (V[j] - sum_{i<j} h_i V_i) * fsc[0] (for
// j = 0 only the scaling: V[0] holds the residual and fsc[0] = 1/beta), and
// in the same read of V form part[blk][i] = V_i . w for i <= j (V_j
// completed) with w = V[j + 1], the operator's output of this step.  The
// column of V_0 .. V_{j-1} is held (HOLD) or reloaded as in updots.
template <int NV, bool HOLD>
__global__ __launch_bounds__(KT) void finish_dots_kernel(Slots sl, double* __restrict__ V, int64_t ldv,
                                                         const double* __restrict__ h,
                                                         const double* __restrict__ fsc, int64_t n,
                                                         double* __restrict__ part, int nblk) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  const int j = bs.jj;
  const int jl = j > 0 ? j - 1 : 0;  // loads past j - 1 re-read this (valid) vector
  V = at(V, bs.ws);
  h = at(h, bs.ws);
  fsc = at(fsc, bs.ws);
  part = at(part, bs.ws);
  const double* __restrict__ w = V + int64_t(j + 1) * ldv;
  __shared__ double red[4 * NV];
  __shared__ double ru[KT / 64];
  __shared__ double hs[NV];
  if (threadIdx.x < NV) hs[threadIdx.x] = int(threadIdx.x) < j ? h[threadIdx.x] : 0.0;
  __syncthreads();
  const double sc = fsc[0];
  double* __restrict__ Vj = V + int64_t(j) * ldv;
  int64_t beg, end;
  chunk_of(n, nblk, beg, end);
  double acc[NV];
  double accu = 0.0;
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  if constexpr (HOLD && NV <= 8) {
    // two elements per trip, as in updots
    for (int64_t e = beg + threadIdx.x; e < end; e += 2 * KT) {
      const int64_t e2 = e + KT < end ? e + KT : e;
      double v0[NV], v1[NV];
      const double we0 = w[e], we1 = w[e2];
      double u0 = Vj[e], u1 = Vj[e2];
#pragma unroll
      for (int i = 0; i < NV; ++i) v0[i] = V[int64_t(i < j ? i : jl) * ldv + e];
#pragma unroll
      for (int i = 0; i < NV; ++i) v1[i] = V[int64_t(i < j ? i : jl) * ldv + e2];
#pragma unroll
      for (int i = 0; i < NV; ++i) u0 -= hs[i] * v0[i];
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += v0[i] * we0;
      u0 *= sc;
      Vj[e] = u0;
      accu += u0 * we0;
      if (e + KT < end) {
#pragma unroll
        for (int i = 0; i < NV; ++i) u1 -= hs[i] * v1[i];
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[i] += v1[i] * we1;
        u1 *= sc;
        Vj[e2] = u1;
        accu += u1 * we1;
      }
    }
  } else
  for (int64_t e = beg + threadIdx.x; e < end; e += KT) {
    const double we = w[e];
    double u = Vj[e];
    if constexpr (HOLD) {
      double v[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] = V[int64_t(i < j ? i : jl) * ldv + e];
#pragma unroll
      for (int i = 0; i < NV; ++i) u -= hs[i] * v[i];
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += v[i] * we;
    } else {
#pragma unroll
      for (int i = 0; i < NV; ++i) u -= hs[i] * V[int64_t(i < j ? i : jl) * ldv + e];
      __asm__ volatile("" ::: "memory");  // compiler fence: reload the column, do not keep it live
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += V[int64_t(i < j ? i : jl) * ldv + e] * we;
    }
    u *= sc;
    Vj[e] = u;
    accu += u * we;
  }
  const double su = block_sum(accu, ru);
  if (threadIdx.x == 0) part[int64_t(blockIdx.x) * HMAX + j] = su;
  block_store<NV>(acc, j, part, red);
}

// out[i] = sum_blk part[blk][i], one block per i, fixed order.
__global__ __launch_bounds__(KT) void reduce_kernel(Slots sl, const double* __restrict__ part, int nblk,
                                                    double* __restrict__ out) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  part = at(part, bs.ws);
  out = at(out, bs.ws);
  __shared__ double red[KT / 64];
  const int i = blockIdx.x;
  double s = 0;
  for (int b = threadIdx.x; b < nblk; b += KT) s += part[int64_t(b) * HMAX + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) out[i] = s;
}

// Close Arnoldi step j: assemble column j of the Hessenberg matrix
// (h1 + h2 from the two Gram-Schmidt passes; below the diagonal the norm of
// w2 = w1 - V h2, which for orthonormal V is sqrt(||w1||^2 - ||h2||^2) since
// h2 = V^T w1), rotate it by the previous Givens rotations, form the new
// rotation, update g, and publish stat = {|g_{j+1}|/||b||, flags, ||w2||,
// 1/||w2||}.  h2[j + 1] holds ||w1||^2.  flags: 1 = non-finite value,
// 2 = ||w2|| negligible (the Krylov space is invariant: the least-squares
// solution is exact).
__global__ void finish_kernel(Slots sl, const double* __restrict__ h1, const double* __restrict__ h2, int k,
                              int jmax, double* __restrict__ H, double* __restrict__ cs, double* __restrict__ sn,
                              double* __restrict__ g, const double* __restrict__ bnorm,
                              double* __restrict__ stat) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  const int j = bs.jj;
  h1 = at(h1, bs.ws);
  h2 = at(h2, bs.ws);
  H = at(H, bs.ws);
  cs = at(cs, bs.ws);
  sn = at(sn, bs.ws);
  g = at(g, bs.ws);
  bnorm = at(bnorm, bs.ws);
  stat = at(stat, bs.ws);
  double* col = H + int64_t(j) * (k + 1);
  double cmax = 0, h2sq = 0;
  for (int i = 0; i <= j; ++i) {
    col[i] = h1[i] + h2[i];
    cmax = fmax(cmax, fabs(col[i]));
    h2sq += h2[i] * h2[i];
  }
  const double hn2 = h2[j + 1] - h2sq;
  const double hn = hn2 > 0 ? sqrt(hn2) : 0.0;
  col[j + 1] = hn;
  int flags = 0;
  if (!isfinite(hn2) || !isfinite(cmax) || j > jmax) flags |= 1;
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
  // the next preconditioner input is w1 / ||w1|| (w1 left in V[j + 1])
  stat[5] = h2[j + 1] > 0 ? 1.0 / sqrt(h2[j + 1]) : 0.0;
  if (!isfinite(stat[0])) {
    flags |= 1;
    stat[1] = double(flags);
  }
  // the slot's own stopping test: a non-finite value discards the cycle; a
  // stopped slot waits at the cycle boundary
  SlotDesc* d = sl.tab + blockIdx.z;
  d->steps += 1;
  if (flags & 1) {
    d->bad = 1;
    d->jj = 0;
    d->live = 0;
    d->edge = 1;
  } else {
    d->jj = j + 1;
    if ((flags & 2) || stat[0] <= d->rtol || j + 1 >= d->limit) {
      d->live = 0;
      d->edge = 1;
    }
  }
}

// beta = ||r|| from partial sums; g = beta e_1; stat[3] = 1/beta, stat[4] = beta.
__global__ __launch_bounds__(KT) void start_cycle_kernel(Slots sl, const double* __restrict__ partn, int nblk,
                                                         double* __restrict__ g, int k, double* __restrict__ stat) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  partn = at(partn, bs.ws);
  if (g) g = at(g, bs.ws);
  stat = at(stat, bs.ws);
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
  // V[0] holds r: the first preconditioner input is r / beta, and the
  // first step's pass 1 scales V[0] in place
  stat[5] = stat[3];
}

// The decision at a cycle boundary, per slot at the edge, in the order of
// the single-solve driver: a non-finite right-hand side, a zero one, a
// breakdown in the cycle, convergence of the true residual, the iteration
// limit, and stagnation (three boundaries in a row that each cut the true
// residual by less than 0.1 %); otherwise a new cycle of at most k steps.
// stat[4] = beta = ||b - L x||, bn[0] = ||b||.
__global__ void decide_kernel(Slots sl, const double* __restrict__ stat, const double* __restrict__ bn, int k) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  stat = at(stat, bs.ws);
  bn = at(bn, bs.ws);
  SlotDesc* d = sl.tab + blockIdx.z;
  const double beta = stat[4];
  const int jj = d->jj;
  d->iters += jj;
  if (jj > 0) d->restarts += 1;
  d->edge = 0;
  d->live = 0;
  d->jj = 0;
  int done = 0, code = RTE_OK;
  if (d->bnorm < 0) {
    const double b = bn[0];
    d->bnorm = b;
    d->prev = INFINITY;
    if (!isfinite(b)) {
      done = 1;
      code = RTE_EINVAL;
    } else if (b == 0.0) {
      d->rel = 0.0;
      done = 2;
    }
  }
  if (!done) {
    d->rel = beta / d->bnorm;
    if (d->bad || !isfinite(beta)) {
      done = 1;
      code = RTE_EBREAKDOWN;
    } else if (d->rel <= d->rtol) {
      done = 1;
    } else if (d->iters >= d->max_iters) {
      done = 1;
      code = RTE_ENOCONV;
    } else {
      if (beta >= d->prev * (1.0 - 1e-3)) {
        if (++d->stall >= 3) {
          done = 1;
          code = RTE_ENOCONV;
        }
      } else {
        d->stall = 0;
      }
    }
  }
  d->bad = 0;
  if (done) {
    d->done = done;
    d->code = code;
    return;
  }
  d->prev = beta;
  const int left = d->max_iters - d->iters;
  d->limit = left < k ? left : k;
  d->live = 1;
}

// Back substitution on the rotated (upper-triangular) Hessenberg matrix.
__global__ void lsq_kernel(Slots sl, const double* __restrict__ H, const double* __restrict__ g, int jj, int k,
                           double* __restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  if (sl.tab) jj = sl.tab[blockIdx.z].jj;
  H = at(H, bs.ws);
  g = at(g, bs.ws);
  y = at(y, bs.ws);
  for (int i = jj - 1; i >= 0; --i) {
    double s = g[i];
    for (int l = i + 1; l < jj; ++l) s -= H[int64_t(l) * (k + 1) + i] * y[l];
    y[i] = s / H[int64_t(i) * (k + 1) + i];
  }
}

// x += sum_i y_i Z_i (Z stored in FP32).
__global__ __launch_bounds__(KT) void xupdate_kernel(Slots sl, double* __restrict__ x,
                                                     const float* __restrict__ Z, int64_t ldz,
                                                     const double* __restrict__ y, int jj, int64_t n) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  if (sl.tab) jj = sl.tab[blockIdx.z].jj;
  if (jj == 0) return;
  x = at(x, bs.ws);
  Z = at(Z, bs.ws);
  y = at(y, bs.ws);
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

__global__ void admit_kernel(SlotDesc* __restrict__ tab, const SlotInit* __restrict__ init, int64_t n,
                             uint64_t off_x, uint64_t off_b) {
  const int z = blockIdx.z;
  if (!init[z].admit) return;
  const uint64_t ws = init[z].d.ws;
  double* __restrict__ x = reinterpret_cast<double*>(ws + off_x);
  double* __restrict__ b = reinterpret_cast<double*>(ws + off_b);
  const double* __restrict__ x0 = reinterpret_cast<const double*>(init[z].x0);
  const double* __restrict__ bs = reinterpret_cast<const double*>(init[z].b);
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x) {
    x[e] = x0 ? x0[e] : 0.0;
    b[e] = bs[e];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) tab[z] = init[z].d;
}

__global__ void emit_kernel(const SlotEmit* __restrict__ em, int64_t n) {
  const int z = blockIdx.z;
  const int mode = em[z].mode;
  if (!mode) return;
  double* __restrict__ out = reinterpret_cast<double*>(em[z].out);
  const double* __restrict__ x = reinterpret_cast<const double*>(em[z].x);
  if (mode == 1) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
      out[e] = x[e];
  } else {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
      out[e] = 0.0;
  }
}

unsigned ew_grid(int64_t n) {
  int64_t g = (n + KT - 1) / KT;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return unsigned(g);
}

}  // namespace

// Partial-sum blocks for a length-n reduction: about 2048 elements per block
// (eight per thread), at most 2048 blocks; depends on n only.
int krylov_blocks(int64_t n) {
  int64_t b = (n + 2047) / 2048;
  if (b < 1) b = 1;
  if (b > 2048) b = 2048;
  return int(b);
}

namespace {
template <int NV>
void dots_go(dim3 g, hipStream_t s, const ProfScope& ps, const Slots& sl, const double* V, int64_t ldv, int nv,
             const double* w, int64_t n, double* part, int nblk) {
  launch_k(dots_kernel<NV>, g, dim3(KT), 0, s, ps, sl, V, ldv, nv, w, n, part, nblk);
}
template <int NV>
void updots_go(dim3 g, hipStream_t s, const ProfScope& ps, const Slots& sl, const double* V, int64_t ldv,
               const double* h, int64_t n, double* part, int nblk) {
  launch_k(updots_kernel<NV, (NV <= 32)>, g, dim3(KT), 0, s, ps, sl, V, ldv, h, n, part, nblk);
}
dim3 z3(unsigned x, const Slots& sl) { return dim3(x, 1, unsigned(sl.count)); }
}  // namespace

void launch_dots(const Slots& sl, const double* V, int64_t ldv, int nv, const double* w, int64_t n, double* part,
                 int nblk, hipStream_t s) {
  RTE_REQUIRE(nv >= 1 && nv <= 64, RTE_EINVAL, "too many basis vectors");
  ProfScope ps(RTE_K_ORTH, s, true);
  ps.key = 1;
  ps.work = 8.0 * double(n) * (nv + 1);
  const dim3 g = z3(unsigned(nblk), sl);
  if (nv <= 4) dots_go<4>(g, s, ps, sl, V, ldv, nv, w, n, part, nblk);
  else if (nv <= 8) dots_go<8>(g, s, ps, sl, V, ldv, nv, w, n, part, nblk);
  else if (nv <= 16) dots_go<16>(g, s, ps, sl, V, ldv, nv, w, n, part, nblk);
  else if (nv <= 32) dots_go<32>(g, s, ps, sl, V, ldv, nv, w, n, part, nblk);
  else dots_go<64>(g, s, ps, sl, V, ldv, nv, w, n, part, nblk);
  RTE_HIP(hipGetLastError());
}

void launch_reduce(const Slots& sl, const double* part, int nblk, int nv, double* out, hipStream_t s) {
  ProfScope ps(RTE_K_ORTH, s, true);
  ps.key = 2;
  launch_k(reduce_kernel, z3(unsigned(nv), sl), dim3(KT), 0, s, ps, sl, part, nblk, out);
  RTE_HIP(hipGetLastError());
}

namespace {
template <int NV>
void fdots_go(dim3 g, hipStream_t s, const ProfScope& ps, const Slots& sl, double* V, int64_t ldv,
              const double* h, const double* fsc, int64_t n, double* part, int nblk) {
  launch_k(finish_dots_kernel<NV, (NV <= 32)>, g, dim3(KT), 0, s, ps, sl, V, ldv, h, fsc, n, part, nblk);
}
}  // namespace

void launch_finish_dots(const Slots& sl, double* V, int64_t ldv, int jmax, const double* h, const double* fsc,
                        int64_t n, double* part, int nblk, hipStream_t s) {
  RTE_REQUIRE(sl.tab != nullptr, RTE_EINVAL, "the Arnoldi step kernels run under a slot table");
  RTE_REQUIRE(jmax >= 0 && jmax <= 63, RTE_EINVAL, "too many basis vectors");
  ProfScope ps(RTE_K_ORTH, s, true);
  ps.key = 3;
  ps.work = 8.0 * double(n) * (jmax + 3);  // V_0..V_{j-1}, V_j read and written, w (j at its bound)
  const dim3 g = z3(unsigned(nblk), sl);
  if (jmax <= 4) fdots_go<4>(g, s, ps, sl, V, ldv, h, fsc, n, part, nblk);
  else if (jmax <= 8) fdots_go<8>(g, s, ps, sl, V, ldv, h, fsc, n, part, nblk);
  else if (jmax <= 16) fdots_go<16>(g, s, ps, sl, V, ldv, h, fsc, n, part, nblk);
  else if (jmax <= 32) fdots_go<32>(g, s, ps, sl, V, ldv, h, fsc, n, part, nblk);
  else fdots_go<64>(g, s, ps, sl, V, ldv, h, fsc, n, part, nblk);
  RTE_HIP(hipGetLastError());
}

void launch_updots(const Slots& sl, const double* V, int64_t ldv, int jmax, const double* h, int64_t n,
                   double* part, int nblk, hipStream_t s) {
  RTE_REQUIRE(sl.tab != nullptr, RTE_EINVAL, "the Arnoldi step kernels run under a slot table");
  RTE_REQUIRE(jmax >= 0 && jmax <= 63, RTE_EINVAL, "too many basis vectors");
  const int nv = jmax + 1;
  ProfScope ps(RTE_K_ORTH, s, true);
  ps.key = 4;
  ps.work = 8.0 * double(n) * (nv + 2);  // V once, w read and written once (j at its bound)
  const dim3 g = z3(unsigned(nblk), sl);
  if (nv <= 4) updots_go<4>(g, s, ps, sl, V, ldv, h, n, part, nblk);
  else if (nv <= 8) updots_go<8>(g, s, ps, sl, V, ldv, h, n, part, nblk);
  else if (nv <= 16) updots_go<16>(g, s, ps, sl, V, ldv, h, n, part, nblk);
  else if (nv <= 32) updots_go<32>(g, s, ps, sl, V, ldv, h, n, part, nblk);
  else updots_go<64>(g, s, ps, sl, V, ldv, h, n, part, nblk);
  RTE_HIP(hipGetLastError());
}

void launch_finish_step(const Slots& sl, const double* h1, const double* h2, int k, int jmax, double* H,
                        double* cs, double* sn, double* g, const double* bnorm, double* stat, hipStream_t s) {
  RTE_REQUIRE(sl.tab != nullptr, RTE_EINVAL, "the Arnoldi step kernels run under a slot table");
  ProfScope ps(RTE_K_ORTH, s, true);
  ps.key = 5;
  launch_k(finish_kernel, z3(1, sl), dim3(64), 0, s, ps, sl, h1, h2, k, jmax, H, cs, sn, g, bnorm, stat);
  RTE_HIP(hipGetLastError());
}

void launch_decide(const Slots& sl, const double* stat, const double* bn, int k, hipStream_t s) {
  RTE_REQUIRE(sl.tab != nullptr, RTE_EINVAL, "the boundary decision runs under a slot table");
  hipLaunchKernelGGL(decide_kernel, z3(1, sl), dim3(64), 0, s, sl, stat, bn, k);
  RTE_HIP(hipGetLastError());
}

void launch_admit(SlotDesc* tab, const SlotInit* init, int count, int64_t n, uint64_t off_x, uint64_t off_b,
                  hipStream_t s) {
  hipLaunchKernelGGL(admit_kernel, dim3(ew_grid(n), 1, unsigned(count)), dim3(KT), 0, s, tab, init, n, off_x,
                     off_b);
  RTE_HIP(hipGetLastError());
}

void launch_emit(const SlotEmit* em, int count, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(emit_kernel, dim3(ew_grid(n), 1, unsigned(count)), dim3(KT), 0, s, em, n);
  RTE_HIP(hipGetLastError());
}

void launch_start_cycle(const Slots& sl, const double* partn, int nblk, double* g, int k, double* stat,
                        hipStream_t s) {
  hipLaunchKernelGGL(start_cycle_kernel, z3(1, sl), dim3(KT), 0, s, sl, partn, nblk, g, k, stat);
  RTE_HIP(hipGetLastError());
}

void launch_lsq(const Slots& sl, const double* H, const double* g, int jj, int k, double* y, hipStream_t s) {
  hipLaunchKernelGGL(lsq_kernel, z3(1, sl), dim3(64), 0, s, sl, H, g, jj, k, y);
  RTE_HIP(hipGetLastError());
}

void launch_xupdate(const Slots& sl, double* x, const float* Z, int64_t ldz, const double* y, int jj, int64_t n,
                    hipStream_t s) {
  hipLaunchKernelGGL(xupdate_kernel, z3(ew_grid(n), sl), dim3(KT), 0, s, sl, x, Z, ldz, y, jj, n);
  RTE_HIP(hipGetLastError());
}

}  // namespace rte

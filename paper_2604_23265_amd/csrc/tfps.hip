// Tailored finite point scheme (Sec. 2.2) on the device: y = A x for the
// midpoint continuity and inflow conditions of eq. (2DTFPS_continuity_cond)
// and eq. (2DTFPS_boundary_cond), r = b - A x, and the solution at the cell
// centres (eq. (2DTFPS_sol)).
//
// The value of cell C's local solution at the midpoint of face f is
// V_f = L_C (e_f (.) x_C): L_C [N x 2N] holds the cell's eigenvectors (one
// table per distinct medium ratio, stored transposed [2N][N] so that lanes
// over directions read coalesced rows), x_C its 2N coefficients and e_f the
// basis functions' exponential factors at that midpoint, exp(sT xi h t) with
// t in {-1, -1/2, 0, 1/2, 1} set by the function's reference edge -- formed
// on the fly from xi and sT.  Per cell that is a [N x 2N] x [2N x 4] product
// whose operand is the cell's own table: the work is bound by reading the
// tables (about one flop per byte in FP64), so it runs on the vector units,
// not the matrix cores.
//
// A block holds 256 / P cells (P = N rounded up to a power of two lanes per
// cell).  Phase 1 forms the 4 x 2N products e_f x_C of its cells in LDS;
// phase 2 has lane m of a cell accumulate row m of the four face values;
// phase 3 adds each face value into the equation rows it enters (its own
// cell's left/bottom row with sign -1, the right/top neighbour's row with sign
// +1, or a boundary row).  Every interior row receives exactly two atomic
// additions onto zero and every boundary row one, so the result is
// independent of their order: fl(fl(0 + a) + b) = fl(a + b) = fl(b + a).
// The residual accumulates the negated contributions the same way and adds
// b afterwards.
#include <algorithm>

#include "common.h"

namespace rte {
namespace {

constexpr int TB = 256;

template <class T>
__device__ inline void atomic_add(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

// exponential factors of basis function k at the left/right/bottom/top face
// midpoints and the centre (f = 0..4)
__device__ inline void factors(double a, int k, int N, double e[5]) {
  const bool xtype = k < N;
  const bool neg = (k - (xtype ? 0 : N)) < N / 2;
  // positions of the lower and upper face relative to the reference edge (units of h)
  const double lo_pos = neg ? 0.0 : -1.0, hi_pos = neg ? 1.0 : 0.0;
  const double lo = exp(a * lo_pos), hi = exp(a * hi_pos), mid = exp(a * 0.5 * (lo_pos + hi_pos));
  if (xtype) {
    e[0] = lo; e[1] = hi; e[2] = mid; e[3] = mid;
  } else {
    e[0] = mid; e[1] = mid; e[2] = lo; e[3] = hi;
  }
  e[4] = mid;
}

template <class TX, class TY, bool RES>
__global__ __launch_bounds__(TB) void tfps_faces_kernel(Slots sl, const TX* __restrict__ x, TY* __restrict__ y,
                                                        const int* __restrict__ bid, const double* __restrict__ sT,
                                                        const uint64_t* __restrict__ tab,
                                                        const int* __restrict__ dsgn, int N, int P, int I,
                                                        double h) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  x = at(x, bs.ws + bs.dx);
  y = at(y, bs.ws + bs.dy);
  bid = at(bid, bs.op);
  sT = at(sT, bs.op);
  tab = at(tab, bs.op);
  dsgn = at(dsgn, bs.op);
  const double* __restrict__ Lt = reinterpret_cast<const double*>(tab[0]);
  const double* __restrict__ xi = reinterpret_cast<const double*>(tab[1]);
  extern __shared__ double wsm[];  // [cpb][4][2N]
  const int K = 2 * N;
  const int cpb = TB / P;
  const int64_t cells = int64_t(I) * I;
  const int64_t c0 = int64_t(blockIdx.x) * cpb;
  for (int idx = threadIdx.x; idx < cpb * K; idx += TB) {
    const int cl = idx / K, k = idx - (idx / K) * K;
    const int64_t c = c0 + cl;
    double e[5] = {0, 0, 0, 0, 0};
    double xv = 0;
    if (c < cells) {
      const int b = bid[c];
      factors(sT[c] * h * xi[size_t(b) * K + k], k, N, e);
      xv = double(x[c * K + k]);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) wsm[(cl * 4 + f) * K + k] = e[f] * xv;
  }
  __syncthreads();
  const int cl = threadIdx.x / P, m = threadIdx.x - (threadIdx.x / P) * P;
  const int64_t c = c0 + cl;
  if (m >= N || c >= cells) return;
  const double* __restrict__ L = Lt + size_t(bid[c]) * K * N;
  const double* w = wsm + cl * 4 * K;
  double v0 = 0, v1 = 0, v2 = 0, v3 = 0;
  for (int k = 0; k < K; ++k) {
    const double l = L[size_t(k) * N + m];
    v0 += l * w[k];
    v1 += l * w[K + k];
    v2 += l * w[2 * K + k];
    v3 += l * w[3 * K + k];
  }
  const int i = int(c % I), j = int(c / I);
  const int sx = dsgn[4 * m], sy = dsgn[4 * m + 1];
  const double sg = RES ? -1.0 : 1.0;
  TY* rowx = y + m;      // + cell * K: the cell's x-face row
  TY* rowy = y + N + m;  // + cell * K: the cell's y-face row
  if (i >= 1) atomic_add(rowx + c * K, TY(-sg * v0));
  else if (sx > 0) atomic_add(rowx + c * K, TY(sg * v0));
  if (i + 1 < I) atomic_add(rowx + (c + 1) * K, TY(sg * v1));
  else if (sx < 0) atomic_add(rowx + (c - i) * K, TY(sg * v1));
  if (j >= 1) atomic_add(rowy + c * K, TY(-sg * v2));
  else if (sy > 0) atomic_add(rowy + c * K, TY(sg * v2));
  if (j + 1 < I) atomic_add(rowy + (c + I) * K, TY(sg * v3));
  else if (sy < 0) atomic_add(rowy + int64_t(i) * K, TY(sg * v3));
}

template <class T>
__global__ void tfps_zero_kernel(Slots sl, T* y, int64_t n) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  y = at(y, bs.ws + bs.dy);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    y[i] = T(0);
}

__global__ void tfps_addb_kernel(Slots sl, double* r, const double* __restrict__ b, int64_t n) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  r = at(r, bs.ws + bs.dy);
  b = at(b, bs.ws);
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    r[i] += b[i];
}

__global__ __launch_bounds__(TB) void tfps_centres_kernel(const double* __restrict__ x, double* __restrict__ psi,
                                                          const int* __restrict__ bid, const double* __restrict__ sT,
                                                          const double* __restrict__ chis,
                                                          const uint64_t* __restrict__ tab, int N, int P, int I,
                                                          double h) {
  const double* __restrict__ Lt = reinterpret_cast<const double*>(tab[0]);
  const double* __restrict__ xi = reinterpret_cast<const double*>(tab[1]);
  extern __shared__ double wsm[];  // [cpb][2N]
  const int K = 2 * N;
  const int cpb = TB / P;
  const int64_t cells = int64_t(I) * I;
  const int64_t c0 = int64_t(blockIdx.x) * cpb;
  for (int idx = threadIdx.x; idx < cpb * K; idx += TB) {
    const int cl = idx / K, k = idx - (idx / K) * K;
    const int64_t c = c0 + cl;
    double v = 0;
    if (c < cells) {
      double e[5];
      factors(sT[c] * h * xi[size_t(bid[c]) * K + k], k, N, e);
      v = e[4] * x[c * K + k];
    }
    wsm[cl * K + k] = v;
  }
  __syncthreads();
  const int cl = threadIdx.x / P, m = threadIdx.x - (threadIdx.x / P) * P;
  const int64_t c = c0 + cl;
  if (m >= N || c >= cells) return;
  const double* __restrict__ L = Lt + size_t(bid[c]) * K * N;
  double v = 0;
  for (int k = 0; k < K; ++k) v += L[size_t(k) * N + m] * wsm[cl * K + k];
  psi[size_t(m) * cells + c] = v + chis[c];
}

int lanes_per_cell(int N) {
  int P = 1;
  while (P < N) P <<= 1;
  return P;
}

unsigned ew_blocks(int64_t n) {
  return unsigned(std::min<int64_t>((n + TB - 1) / TB, 4096));
}

template <class TX, class TY, bool RES>
void tfps_go(const Target& T, const void* x, void* y, const double* b, hipStream_t s, const ProfScope& ps) {
  const Operator& op = *T.op;
  const int N = op.ndir, P = lanes_per_cell(N), cpb = TB / P;
  const int64_t n = op.n;
  const dim3 gz(ew_blocks(n), 1, unsigned(T.sl.count));
  hipLaunchKernelGGL(tfps_zero_kernel<TY>, gz, dim3(TB), 0, s, T.sl, static_cast<TY*>(y), n);
  const dim3 g(unsigned((op.cells + cpb - 1) / cpb), 1, unsigned(T.sl.count));
  const size_t lds = size_t(cpb) * 4 * 2 * N * sizeof(double);
  launch_k(tfps_faces_kernel<TX, TY, RES>, g, dim3(TB), uint32_t(lds), s, ps, T.sl, static_cast<const TX*>(x),
           static_cast<TY*>(y), T.arr.tf_bid, T.arr.sT64, T.arr.tf_tab, T.arr.dsgn, N, P, op.nx, op.h);
  if (RES)
    hipLaunchKernelGGL(tfps_addb_kernel, gz, dim3(TB), 0, s, T.sl, static_cast<double*>(y), b, n);
  RTE_HIP(hipGetLastError());
}

}  // namespace

void launch_tfps_apply(const Target& T, const void* x, int tin, void* y, int tout, const double* b,
                       hipStream_t s) {
  const Operator& op = *T.op;
  RTE_REQUIRE(op.scheme == RTE_SCHEME_TFPS, RTE_EINVAL, "not a TFPS operator");
  const int N = op.ndir;
  // algorithmic bytes: x and y once, each basis table once, per cell its basis index and sT
  const double esz[2] = {4.0, 8.0};
  const double tables = double(op.nbasis) * (2.0 * N * N + 2.0 * N) * 8.0;
  if (b) {
    RTE_REQUIRE(tin == 1 && tout == 1, RTE_EINVAL, "residual is FP64 only");
    ProfScope ps(RTE_K_RESIDUAL, s, true);
    ps.work = 24.0 * double(op.n) + tables + 12.0 * double(op.cells);
    tfps_go<double, double, true>(T, x, y, b, s, ps);
    return;
  }
  ProfScope ps(RTE_K_APPLY, s, true);
  ps.work = (esz[tin] + esz[tout]) * double(op.n) + tables + 12.0 * double(op.cells);
  if (tin == 1 && tout == 1) tfps_go<double, double, false>(T, x, y, nullptr, s, ps);
  else if (tin == 0 && tout == 1) tfps_go<float, double, false>(T, x, y, nullptr, s, ps);
  else if (tin == 0 && tout == 0) tfps_go<float, float, false>(T, x, y, nullptr, s, ps);
  else tfps_go<double, float, false>(T, x, y, nullptr, s, ps);
}

void launch_operator(const Target& T, const void* x, int tin, void* y, int tout, const double* b, bool fp64,
                     hipStream_t s) {
  if (T.op->scheme == RTE_SCHEME_TFPS)
    launch_tfps_apply(T, x, tin, y, tout, b, s);  // computed in FP64 whatever the vectors' types
  else
    launch_apply(T, x, tin, y, tout, b, fp64, s);
}

void launch_tfps_centres(const Target& T, const double* x, double* psi, hipStream_t s) {
  const Operator& op = *T.op;
  RTE_REQUIRE(op.scheme == RTE_SCHEME_TFPS && !T.sl.tab, RTE_EINVAL, "centre values: one TFPS operator");
  const int N = op.ndir, P = lanes_per_cell(N), cpb = TB / P;
  const dim3 g(unsigned((op.cells + cpb - 1) / cpb));
  const size_t lds = size_t(cpb) * 2 * N * sizeof(double);
  hipLaunchKernelGGL(tfps_centres_kernel, g, dim3(TB), uint32_t(lds), s, x, psi, T.arr.tf_bid, T.arr.sT64,
                     T.arr.tf_chis, T.arr.tf_tab, N, P, op.nx, op.h);
  RTE_HIP(hipGetLastError());
}

}  // namespace rte

// ------------------------------------------------------------- ATFPS ---
// The compressed system, the layer reconstruction and the filtered loss of
// Sec. 2.3 / Sec. 3.4 are sparse linear maps plus constants, assembled on the
// host.  A wave takes a row: lanes stride over its nonzeros, a wave-level
// sum in fixed order combines them (rows hold at most 4 N nonzeros), so every
// result is reproducible.
namespace rte {
namespace {

__global__ __launch_bounds__(256) void csr_kernel(int64_t nrows, const int64_t* __restrict__ ptr,
                                                  const int64_t* __restrict__ col, const double* __restrict__ val,
                                                  const double* __restrict__ x, const double* __restrict__ c,
                                                  int sub, double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t r = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (r >= nrows) return;
  double s = 0;
  for (int64_t e = ptr[r] + lane; e < ptr[r + 1]; e += 64) s += val[e] * x[col[e]];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
  if (lane == 0) {
    const double cv = c ? c[r] : 0.0;
    y[r] = sub ? cv - s : s + cv;
  }
}

// Sum of squares in two stages with a fixed assignment: block b of the first
// stage owns elements [b chunk, (b + 1) chunk) and writes its partial; one
// block then adds the partials in block order.  The result does not depend
// on scheduling.
__global__ __launch_bounds__(256) void sumsq_kernel(const double* __restrict__ v, int64_t n, int64_t chunk,
                                                    double* __restrict__ part) {
  __shared__ double w4[4];
  const int64_t b0 = int64_t(blockIdx.x) * chunk, b1 = b0 + chunk < n ? b0 + chunk : n;
  double s = 0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) s += v[i] * v[i];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
  if ((threadIdx.x & 63) == 0) w4[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((w4[0] + w4[1]) + w4[2]) + w4[3];
}

__global__ __launch_bounds__(256) void norm2_kernel(const double* __restrict__ part, int nb, double* out) {
  __shared__ double w4[4];
  double s = 0;
  for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
  if ((threadIdx.x & 63) == 0) w4[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = sqrt(((w4[0] + w4[1]) + w4[2]) + w4[3]);
}

}  // namespace

void launch_csr(const DevCsr& A, const double* x, const double* c, bool sub, double* y, hipStream_t s) {
  if (A.nrows == 0) return;
  hipLaunchKernelGGL(csr_kernel, dim3(unsigned((A.nrows + 3) / 4)), dim3(256), 0, s, A.nrows, A.ptr, A.col, A.val,
                     x, c, sub ? 1 : 0, y);
  RTE_HIP(hipGetLastError());
}

void launch_norm2(const double* v, int64_t n, double* part, double* out, hipStream_t s) {
  const int64_t chunk = std::max<int64_t>(4096, (n + kNorm2Parts - 1) / kNorm2Parts);
  const int nb = int(std::max<int64_t>(1, (n + chunk - 1) / chunk));
  hipLaunchKernelGGL(sumsq_kernel, dim3(unsigned(nb)), dim3(256), 0, s, v, n, chunk, part);
  hipLaunchKernelGGL(norm2_kernel, dim3(1), dim3(256), 0, s, part, nb, out);
  RTE_HIP(hipGetLastError());
}

}  // namespace rte

// Cell-wise Block-Jacobi preconditioner, the classical comparator of the
// paper's experiments (Sec. 4).
#include "common.h"

// ------------------------------------------------------- Block-Jacobi ---
// z_c = B_c^{-1} v_c for every cell c, with B_c the N x N block of L that
// couples the cell's directions:
//   B_c = diag_m(sum_a |u_{m,a}| / h) + sT_c (I - S) + sA_c S
// (sT - sS = sA: the cancellation-free form the apply uses).  B_c is
// diagonally dominant (row sums of S are 1), so Gaussian elimination needs
// no pivoting.  A group of NB lanes solves one cell: lane i holds row i of
// B_c (S row i kept in registers across cells) and v_i; the pivot row is
// broadcast with lane shuffles.  Rows i >= N are identity padding.  The
// block stages v for 64 cells in LDS (coalesced), each wave solves 16 of
// them, and the results leave through the same LDS tile.
namespace rte {
namespace {

template <int NB>
__global__ __launch_bounds__(256) void block_jacobi_kernel(Slots sl, const double* __restrict__ v,
                                                           const double* __restrict__ vs,
                                                           const float* __restrict__ sT,
                                                           const float* __restrict__ sA,
                                                           const float* __restrict__ S,
                                                           const float* __restrict__ dc, float* __restrict__ z,
                                                           int N, int cells) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  v = at(v, bs.ws + bs.dx);
  z = at(z, bs.ws + bs.dy);
  const double vsc = vs ? at(vs, bs.ws)[0] : 1.0;
  sT = at(sT, bs.op);
  sA = at(sA, bs.op);
  S = at(S, bs.op);
  dc = at(dc, bs.op);
  extern __shared__ float xs[];  // [N][64]
  const int c0 = int(blockIdx.x) * 64;
  for (int idx = threadIdx.x; idx < N * 64; idx += 256) {
    const int m = idx >> 6, cc = c0 + (idx & 63);
    const double val = v[int64_t(m) * cells + (cc < cells ? cc : cells - 1)];
    xs[idx] = cc < cells ? float(val * vsc) : 0.f;
  }
  __syncthreads();
  constexpr int G = 64 / NB;  // cells per wave per pass
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int i = lane % NB;            // row of B_c
  const int base = lane - i;          // first lane of the group
  const int grp = lane / NB;
  const bool real = i < N;
  const int ic = real ? i : N - 1;
  float srow[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) srow[j] = (real && j < N) ? S[ic * N + j] : 0.f;
  const float di = dc[4 * ic + 3];
  for (int pass = 0; pass < 16 / G; ++pass) {
    const int cl = wave * 16 + pass * G + grp;   // cell within the tile
    const int c = c0 + cl;
    const int cc = c < cells ? c : cells - 1;
    const float t = sT[cc], a_ = sA[cc];
    float a[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const float e = j == i ? 1.f : 0.f;
      a[j] = real ? t * (e - srow[j]) + a_ * srow[j] + e * di : e;
    }
    float r = real ? xs[i * 64 + cl] : 0.f;
    // forward elimination
#pragma unroll
    for (int k = 0; k < NB - 1; ++k) {
      const float pkk = __shfl(a[k], base + k, 64);
      const float l = i > k ? a[k] / pkk : 0.f;
#pragma unroll
      for (int j = k + 1; j < NB; ++j) a[j] -= l * __shfl(a[j], base + k, 64);
      r -= l * __shfl(r, base + k, 64);
    }
    // back substitution: lane k's unknown is r_k / a_kk once rows below are done
    float x = 0.f;
#pragma unroll
    for (int k = NB - 1; k >= 0; --k) {
      const float xk = __shfl(r / a[k], base + k, 64);
      if (i == k) x = xk;
      if (i < k) r -= a[k] * xk;
    }
    if (real) xs[i * 64 + cl] = x;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < N * 64; idx += 256) {
    const int m = idx >> 6, cc = c0 + (idx & 63);
    if (cc < cells) z[int64_t(m) * cells + cc] = xs[idx];
  }
}

// Block-Jacobi for 65 to 112 directions (the 3D sphere sets): one wave per
// cell, the cell's N x N block in LDS column by column (entry (i, j) at
// j N + i, so the lanes' rows of one column are consecutive words), Gaussian
// elimination without pivoting as above, lane l owning rows l and l + 64.
// Each elimination step reads the pivot row as broadcasts and updates the
// trailing block; back substitution walks the columns from the last.
__global__ __launch_bounds__(64) void block_jacobi_wide_kernel(Slots sl, const double* __restrict__ v,
                                                               const double* __restrict__ vs,
                                                               const float* __restrict__ sT,
                                                               const float* __restrict__ sA,
                                                               const float* __restrict__ S,
                                                               const float* __restrict__ dc, float* __restrict__ z,
                                                               int N, int cells) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  v = at(v, bs.ws + bs.dx);
  z = at(z, bs.ws + bs.dy);
  const double vsc = vs ? at(vs, bs.ws)[0] : 1.0;
  sT = at(sT, bs.op);
  sA = at(sA, bs.op);
  S = at(S, bs.op);
  dc = at(dc, bs.op);
  extern __shared__ float Am[];  // [N][N], column-major
  const int c = int(blockIdx.x);
  const int lane = int(threadIdx.x);
  const float t = sT[c], a_ = sA[c];
  const int i0 = lane, i1 = lane + 64;
  const bool has1 = i1 < N;
  // B_c = diag(sum_a |u_a| / h) + sT (I - S) + sA S
  for (int j = 0; j < N; ++j) {
    {
      const float e = i0 == j ? 1.f : 0.f;
      const float sij = S[i0 * N + j];
      Am[j * N + i0] = t * (e - sij) + a_ * sij + e * dc[4 * i0 + 3];
    }
    if (has1) {
      const float e = i1 == j ? 1.f : 0.f;
      const float sij = S[i1 * N + j];
      Am[j * N + i1] = t * (e - sij) + a_ * sij + e * dc[4 * i1 + 3];
    }
  }
  float r0 = float(v[int64_t(i0) * cells + c] * vsc);
  float r1 = has1 ? float(v[int64_t(i1) * cells + c] * vsc) : 0.f;
  __syncthreads();
  // forward elimination: rows below the pivot take l = a_ik / a_kk times its row
  for (int k = 0; k < N - 1; ++k) {
    const float pkk = Am[k * N + k];
    const float rk = __shfl(k < 64 ? r0 : r1, k & 63, 64);
    const float l0 = i0 > k ? Am[k * N + i0] / pkk : 0.f;
    const float l1 = has1 && i1 > k ? Am[k * N + i1] / pkk : 0.f;
    for (int j = k + 1; j < N; ++j) {
      const float pj = Am[j * N + k];
      if (i0 > k) Am[j * N + i0] -= l0 * pj;
      if (has1 && i1 > k) Am[j * N + i1] -= l1 * pj;
    }
    r0 -= l0 * rk;
    r1 -= l1 * rk;
    __syncthreads();
  }
  // back substitution
  float x0 = 0.f, x1 = 0.f;
  for (int k = N - 1; k >= 0; --k) {
    const float rk = __shfl(k < 64 ? r0 : r1, k & 63, 64);
    const float xk = rk / Am[k * N + k];
    if (i0 == k) x0 = xk;
    if (i1 == k) x1 = xk;
    if (i0 < k) r0 -= Am[k * N + i0] * xk;
    if (has1 && i1 < k) r1 -= Am[k * N + i1] * xk;
  }
  z[int64_t(i0) * cells + c] = x0;
  if (has1) z[int64_t(i1) * cells + c] = x1;
}

}  // namespace

void launch_block_jacobi(const Target& T, const double* v, const double* vscale, float* z, hipStream_t s) {
  const Operator& op = *T.op;
  RTE_REQUIRE(op.ndir <= RTE_BJ_MAX_DIRS, RTE_EINVAL, "Block-Jacobi supports up to 112 directions");
  ProfScope ps(RTE_K_PRECOND, s);
  if (op.ndir > 64) {
    const OpArrays& A = T.arr;
    hipLaunchKernelGGL(block_jacobi_wide_kernel, dim3(unsigned(op.cells), 1, unsigned(T.sl.count)), dim3(64),
                       size_t(op.ndir) * op.ndir * sizeof(float), s, T.sl, v, vscale, A.sT32, A.sA32, A.S32, A.dc32,
                       z, op.ndir, int(op.cells));
    RTE_HIP(hipGetLastError());
    return;
  }
  const dim3 grid(unsigned((op.cells + 63) / 64), 1, unsigned(T.sl.count));
  const size_t lds = size_t(op.ndir) * 64 * sizeof(float);
  const OpArrays& A = T.arr;
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, T.sl, v, vscale, A.sT32, A.sA32, A.S32, A.dc32, z, op.ndir,
                       int(op.cells));
  };
  if (op.ndir <= 16)
    go(block_jacobi_kernel<16>);
  else if (op.ndir <= 32)
    go(block_jacobi_kernel<32>);
  else
    go(block_jacobi_kernel<64>);
  RTE_HIP(hipGetLastError());
}

}  // namespace rte

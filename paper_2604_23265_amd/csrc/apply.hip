// Discrete-ordinates operator apply (eq. (DORTE_2d), step-upwind finite
// volumes): y = L x or y = b - L x, fused streaming + collision + scatter.
//
// Four kernels: apply_mfma_kernel (below) for the FP32 apply with 32, 64 or
// 96 directions, the scatter on the BF16 matrix cores as a three-term split
// product with FP32 accuracy; apply64_mfma_kernel (below) for the FP64 apply
// and residual with 16, 32, 64 or 96 directions, the scatter on the FP64
// matrix cores; apply_slot_kernel (below) for the other FP32 applies, one
// direction slot per wave; and apply_kernel for the FP64 apply and residual
// with other direction counts, described here.
//
// Layout: x, y direction-major [N][cells].  A 256-thread block owns TL
// consecutive cells (64, or 16 for more than 64 directions) and all N
// directions.  The block stages x[:, tile] in LDS (rows of TL cells per
// direction); each thread then owns one cell and the directions d,
// d + 256/TL, ...: the scatter sum_n S_mn x_n reads S from LDS and reuses
// each x_n read for all of the thread's directions; the upwind neighbours
// come from global memory (the same or an adjacent row, cached) and are
// requested before the scatter loop so their latency overlaps it.
// Collision uses the cancellation-free form sT (x - Sx) + sA Sx.
#include <algorithm>
#include <cstdlib>

#include "common.h"

namespace rte {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t v2u __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

// LDS of the vector apply: the x tile, plus S when both fit in kApplyLds (the
// default limit of a launch); else, for 16-cell tiles, S in chunks of
// apply_s_chunk columns.  S rows are padded by one element for 16-cell tiles
// (four direction slots per wave read four rows at once) and not for 64-cell
// tiles, whose reads of S are the same for the whole wave
constexpr int kApplyLds = 64 * 1024;
__host__ __device__ inline int apply_s_chunk(int N, int tile, int esz) {
  const int kc = (kApplyLds / esz - N * tile) / N - 1;
  return kc < 32 ? kc : 32;
}

// A block of NT threads (256; 512 for FP64) owns TL consecutive cells:
// thread t -> cell t % TL, direction slot t / TL (NT / TL slots).  TL = 64
// (one slot per wave) for up to 64 directions, TL = 16 beyond.

// Thread (cell c, slot d) computes directions m = d, d + NT / TL, ... (< N,
// at most DPT of them).  The block stages x[:, tile] (and S when it fits) in
// LDS; the scatter sum_n S_mn x_n then reuses each x_n read for all of the
// thread's directions.  Upwind neighbours are requested before the scatter.
template <class T, class TI, class TO, bool RES, bool LDS_S, int DPT, int TL, int NT>
__global__ __launch_bounds__(NT) void apply_kernel(Slots sl, const TI* __restrict__ x, TO* __restrict__ y,
                                                    const double* __restrict__ b,
                                                    const T* __restrict__ sT, const T* __restrict__ sA,
                                                    const T* __restrict__ S, const T* __restrict__ dc,
                                                    const int* __restrict__ sg, int N, int nx, int ny,
                                                    int nz, int cells) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  x = at(x, bs.ws + bs.dx);
  y = at(y, bs.ws + bs.dy);
  if (RES) b = at(b, bs.ws);
  sT = at(sT, bs.op);
  sA = at(sA, bs.op);
  S = at(S, bs.op);
  dc = at(dc, bs.op);
  sg = at(sg, bs.op);
  constexpr int TILE = TL;
  constexpr int DSLOTS = NT / TL;
  extern __shared__ char smem[];
  T* xs = reinterpret_cast<T*>(smem);       // [N][TILE]
  T* Ss = xs + N * TILE;                    // [N][ldS]
  const int ldS = TILE == 64 ? N : N + 1;
  const int cl = threadIdx.x & (TILE - 1);
  // with one slot per wave (TL = 64) the slot is wave-uniform: make it a
  // scalar so the per-direction branches and loads stay scalar
  const int slot = TILE == 64 ? __builtin_amdgcn_readfirstlane(int(threadIdx.x) / TILE) : int(threadIdx.x) / TILE;
  const int c0 = int(blockIdx.x) * TILE;
  if (LDS_S) {
    for (int idx = threadIdx.x; idx < N * N; idx += NT) {
      const int r = idx / N;
      Ss[r * ldS + (idx - r * N)] = S[idx];
    }
  }
#pragma unroll 4
  for (int idx = threadIdx.x; idx < N * TILE; idx += NT) {
    const int m = idx / TILE, l = idx - m * TILE;
    const int cc = c0 + l;
    const T v = T(x[int64_t(m) * cells + (cc < cells ? cc : cells - 1)]);  // clamped: no branch around the load
    xs[idx] = cc < cells ? v : T(0);
  }
  __syncthreads();
  // cells past the end compute on the last cell and store nothing: every
  // thread reaches the chunked scatter's barriers
  const bool live = c0 + cl < cells;
  const int c = live ? c0 + cl : cells - 1;
  const int rr = c / nx;
  const int i = c - rr * nx;
  const int k = rr / ny;
  const int j = rr - k * ny;
  const int pos[3] = {i, j, k};
  const int ext[3] = {nx, ny, nz};
  const int stride[3] = {1, nx, nx * ny};
  const T st = sT[c], sa = sA[c];
  // Upwind neighbours of every direction this thread owns, requested
  // together: addresses are clamped to a valid element and a neighbour
  // outside the grid (the inflow, carried by b) is zeroed afterwards, so no
  // branch separates the loads.
  T xc[DPT], str[DPT], acc[DPT];
  T xnb[DPT][3];
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int m = slot + DSLOTS * q;
    const int mc = m < N ? m : N - 1;
    const int64_t o = int64_t(mc) * cells + c;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a == 2 && nz == 1) {
        xnb[q][a] = T(0);
        continue;
      }
      const int sgn = sg[4 * mc + a];
      const int p = pos[a] - sgn;
      const bool inb = p >= 0 && p < ext[a];
      const T v = T(x[inb ? o - sgn * stride[a] : o]);
      xnb[q][a] = inb ? v : T(0);
    }
  }
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int m = slot + DSLOTS * q;
    const int mc = m < N ? m : N - 1;
    xc[q] = xs[mc * TILE + cl];
    acc[q] = T(0);
    T sacc = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) sacc += dc[4 * mc + a] * (xc[q] - xnb[q][a]);
    str[q] = sacc;
  }
  // the scatter runs every one of the thread's DPT direction slots, past N on
  // the last direction's row (stored nowhere), so its loop has no branches:
  // a guard per product became a scalar branch around each LDS read
  int mrow[DPT];
#pragma unroll
  for (int q = 0; q < DPT; ++q) mrow[q] = slot + DSLOTS * q < N ? slot + DSLOTS * q : N - 1;
  if constexpr (!LDS_S && TILE < 64) {
    // S does not fit beside the tile and a wave holds four direction slots,
    // so global reads of S would gather four rows per load: S passes
    // through LDS in chunks of KC columns (rows padded by one element), KC
    // the widest up to 32 that keeps tile and chunk within the launch's LDS
    const int KC = apply_s_chunk(N, TILE, int(sizeof(T)));
    T* Sc = xs + N * TILE;  // [N][KC + 1]
    for (int n0 = 0; n0 < N; n0 += KC) {
      const int kc = N - n0 < KC ? N - n0 : KC;
      if (n0 > 0) __syncthreads();  // the previous chunk is consumed
      for (int idx = threadIdx.x; idx < N * kc; idx += NT) {
        const int r = idx / kc, cc = idx - r * kc;
        Sc[r * (KC + 1) + cc] = S[r * N + n0 + cc];
      }
      __syncthreads();
      for (int n = 0; n < kc; ++n) {
        const T xv = xs[(n0 + n) * TILE + cl];
#pragma unroll
        for (int q = 0; q < DPT; ++q) acc[q] += Sc[mrow[q] * (KC + 1) + n] * xv;
      }
    }
  } else {
#pragma unroll 4
    for (int n = 0; n < N; ++n) {
      const T xv = xs[n * TILE + cl];
#pragma unroll
      for (int q = 0; q < DPT; ++q) acc[q] += (LDS_S ? Ss[mrow[q] * ldS + n] : S[mrow[q] * N + n]) * xv;
    }
  }
  if (!live) return;
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int m = slot + DSLOTS * q;
    if (m >= N) break;
    const int64_t o = int64_t(m) * cells + c;
    const T val = str[q] + st * (xc[q] - acc[q]) + sa * acc[q];
    if (RES)
      y[o] = TO(b[o] - double(val));
    else
      y[o] = TO(val);
  }
}

// Tile of block x when consecutive tiles should share an L2: the
// dispatcher deals workgroups to the eight XCDs round-robin by linear id
// (x % 8 when the grid's x extent is a multiple of 8), so tile
// (x % 8) (T / 8) + x / 8 gives XCD k the contiguous tiles
// [k T / 8, (k + 1) T / 8), and the upwind neighbour rows a tile reads from
// the tiles beside it are mostly in its own L2 instead of another XCD's.
__device__ inline int xcd_tile(int x, int T) { return (T & 7) ? x : (x & 7) * (T >> 3) + (x >> 3); }

// FP32 apply with one direction slot per wave (up to 128 directions): a
// block takes TPB tiles of 64 consecutive cells in turn, lane = cell, wave
// w = directions w, w + 4, ... (at most DPT of them).  The scatter's matrix
// entries are then the same for the whole wave.  With LS (up to 8
// directions per wave) the block stages the slot-packed S in LDS once, one
// vector load per thread, and the scatter reads it with broadcast LDS
// reads: scalar loads of S had to be waited for every two directions and
// serialised the scatter.  Beyond that S comes from scalar loads.  The
// per-direction upwind signs and coefficients and the cell's sigma values
// are requested before any address that uses them, so the upwind
// neighbours are requested together; they are read at clamped addresses and
// zeroed outside the grid.
template <class TO, int DPT, bool D3, bool LS, int TPB>
__global__ __launch_bounds__(256) void apply_slot_kernel(Slots sl, const float* __restrict__ x, TO* __restrict__ y,
                                                         const float* __restrict__ sT, const float* __restrict__ sA,
                                                         const float* __restrict__ Sp, const float* __restrict__ dc,
                                                         const int* __restrict__ sg, int N, int nx, int ny, int nz,
                                                         int cells) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  x = at(x, bs.ws + bs.dx);
  y = at(y, bs.ws + bs.dy);
  sT = at(sT, bs.op);
  sA = at(sA, bs.op);
  Sp = at(Sp, bs.op);
  dc = at(dc, bs.op);
  sg = at(sg, bs.op);
  constexpr int NA = D3 ? 3 : 2;
  extern __shared__ float xs[];  // [N][64] x tile; with LS then S as [4][N][DPT]
  float* ss = xs + N * 64;
  const int lane = threadIdx.x & 63;
  const int slot = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  int sgn[DPT][NA];
  float dcv[DPT][NA];
#pragma unroll
  for (int q = 0; q < DPT; ++q) {
    const int m = slot + 4 * q;
    const int mc = m < N ? m : N - 1;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      sgn[q][a] = sg[4 * mc + a];
      dcv[q][a] = dc[4 * mc + a];
    }
  }
  if constexpr (LS) {
    const int ns = 4 * N * DPT;  // a multiple of 4
    for (int i = 4 * int(threadIdx.x); i < ns; i += 4 * 256)
      *reinterpret_cast<v4f*>(ss + i) = *reinterpret_cast<const v4f*>(Sp + i);
  }
  // the block's TPB tiles of 64 cells, one after another (S staged once)
  const int ntile = (cells + 63) / 64;
  const int tb = xcd_tile(int(blockIdx.x), int(gridDim.x)) * TPB;
  for (int tt = 0; tt < TPB; ++tt) {
    const int tile = tb + tt;
    if (tile >= ntile) break;  // uniform over the block
    if (tt > 0) __syncthreads();  // the previous tile's reads of xs are done
    const int c = tile * 64 + lane;
    const int cc = c < cells ? c : cells - 1;
    const float st = sT[cc], sa = sA[cc];
    // x[:, tile]: this thread's rows are its own directions
    float xown[DPT];
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int m = slot + 4 * q;
      const float v = x[int64_t(m < N ? m : N - 1) * cells + cc];
      xown[q] = c < cells ? v : 0.f;
    }
    const int rr = cc / nx;
    const int i = cc - rr * nx;
    const int k = rr / ny;
    const int j = rr - k * ny;
    const int pos[3] = {i, j, k};
    const int ext[3] = {nx, ny, nz};
    const int stride[3] = {1, nx, nx * ny};
    float xnb[DPT][NA];
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int m = slot + 4 * q;
      const int mc = m < N ? m : N - 1;
      const int64_t o = int64_t(mc) * cells + cc;
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        const int p = pos[a] - sgn[q][a];
        const bool inb = p >= 0 && p < ext[a];
        const float v = x[inb ? o - sgn[q][a] * stride[a] : o];
        xnb[q][a] = inb ? v : 0.f;
      }
    }
#pragma unroll
    for (int q = 0; q < DPT; ++q) {
      const int m = slot + 4 * q;
      if (m < N) xs[m * 64 + lane] = xown[q];
    }
    __syncthreads();
    float acc[DPT];
#pragma unroll
    for (int q = 0; q < DPT; ++q) acc[q] = 0.f;
    if constexpr (LS) {
      const float* sp = ss + slot * N * DPT;
#pragma unroll 4
      for (int n = 0; n < N; ++n) {
        const float xv = xs[n * 64 + lane];
#pragma unroll
        for (int q = 0; q < DPT; ++q) acc[q] += sp[n * DPT + q] * xv;
      }
    } else {
      // DPT scalar registers per direction n; four directions per wait up to
      // DPT = 16 (64 SGPRs), two beyond
      const float* __restrict__ sp = Sp + slot * N * DPT;
#pragma unroll(DPT <= 16 ? 4 : 2)
      for (int n = 0; n < N; ++n) {
        const float xv = xs[n * 64 + lane];
#pragma unroll
        for (int q = 0; q < DPT; ++q) acc[q] += sp[n * DPT + q] * xv;
      }
    }
    if (c < cells) {
#pragma unroll
      for (int q = 0; q < DPT; ++q) {
        const int m = slot + 4 * q;
        if (m >= N) break;
        const float xc = xown[q];
        float str = 0.f;
#pragma unroll
        for (int a = 0; a < NA; ++a) str += dcv[q][a] * (xc - xnb[q][a]);
        const float val = str + st * (xc - acc[q]) + sa * acc[q];
        y[int64_t(m) * cells + c] = TO(val);
      }
    }
  }
}

template <class TO, bool D3>
void go_slot(const Target& Tg, const void* x, void* y, hipStream_t s, const ProfScope& ps) {
  const Operator& op = *Tg.op;
  const OpArrays& A = Tg.arr;
  const int dpt = slot_budget(op.ndir);
  const size_t lds_x = size_t(op.ndir) * 64 * sizeof(float);
  const size_t lds_s = size_t(4) * op.ndir * dpt * sizeof(float);  // slot-packed S
  // S in LDS where its staging (4 N DPT floats per block) is at most half of
  // the block's x tile: up to 32 directions.  With more directions the
  // staging and the LDS it holds cost more than the scalar loads it saves
  // (measured at 64 directions, with one and with four tiles per block).
  const bool ls = dpt <= 8 && lds_x + lds_s <= 64 * 1024;
  const size_t lds = ls ? lds_x + lds_s : lds_x;
  constexpr int TPB_LS = 1;
  const int64_t ntile = (op.cells + 63) / 64;
  const dim3 grid(unsigned(ls ? (ntile + TPB_LS - 1) / TPB_LS : ntile), 1, unsigned(Tg.sl.count));
  auto launch = [&](auto kern) {
    launch_k(kern, grid, dim3(256), uint32_t(lds), s, ps, Tg.sl, static_cast<const float*>(x), static_cast<TO*>(y),
             A.sT32, A.sA32, A.Sp32, A.dc32, static_cast<const int*>(A.dsgn), op.ndir, op.nx, op.ny, op.nz,
             int(op.cells));
  };
  auto pick = [&](auto ls_tag) {
    constexpr bool LS = decltype(ls_tag)::value;
    constexpr int TPB = LS ? TPB_LS : 1;
    switch (dpt) {
      case 1: launch(apply_slot_kernel<TO, 1, D3, LS, TPB>); break;
      case 2: launch(apply_slot_kernel<TO, 2, D3, LS, TPB>); break;
      case 4: launch(apply_slot_kernel<TO, 4, D3, LS, TPB>); break;
      case 8: launch(apply_slot_kernel<TO, 8, D3, LS, TPB>); break;
      case 16: launch(apply_slot_kernel<TO, 16, D3, LS, TPB>); break;
      case 24: launch(apply_slot_kernel<TO, 24, D3, LS, TPB>); break;
      default: launch(apply_slot_kernel<TO, 32, D3, LS, TPB>); break;
    }
  };
  if (ls)
    pick(std::true_type{});
  else
    pick(std::false_type{});
  RTE_HIP(hipGetLastError());
}

// FP32 apply with the scatter on the matrix cores, for N of 32, 64 or 96
// and whole 64-cell tiles: the block has N / 16 waves and wave w owns
// directions 16 w .. 16 w + 15 of each tile.  The scatter (S x)^T for them
// is a [16 x N] x [N x 16] product per 16 cells; the D layout (direction
// 4 (l / 16) + r, cell l % 16) gives each group of 16 lanes 16 consecutive
// cells of one direction, so the streaming part reads and writes coalesced
// rows.  A block walks several tiles (the XCD running it takes a contiguous
// range) and requests the next tile's x into registers before the current
// tile's work.
//
// The product is a three-term bfloat16 split on the BF16 matrix cores
// (16x16x32, sixteen times the FP32 matrix rate):
// x = x0 + x1 + x2 and S = S0 + S1 + S2, each term the bfloat16 rounding of
// what the previous ones leave, so the three terms hold 24 bits of the value
// and leave at most 2^-27 of it.  S x is accumulated in FP32 from the six
// products Si xj with i + j <= 2, per k-step in the order S0 x2, S1 x1, S0 x1,
// S2 x0, S1 x0, S0 x0 (the small ones first); the three dropped products are
// below 2^-26 of |S| |x|, under FP32 rounding.  The block splits the x tile once,
// into three bfloat16 planes [cell][direction] (rows padded by 8, and
// permuted so that both the 16-byte fragment reads of 16 cells and the
// 8-byte staging stores hit every bank equally); each wave splits its rows
// of S once.
//
// ROW (64 divides nx, so a tile is a segment of one grid row): the block
// also stages the tile in FP32, one LDS row per direction with the end
// cells' x-neighbours as halo (zero outside the domain), so x at the lane's
// cells and its upwind x-neighbour are LDS reads; the y / z neighbours are
// loads at per-lane byte offsets fixed for the launch (the own cell where
// the upwind one leaves the domain, its coefficient then zero), requested
// before the scatter and used after it.  Otherwise the streaming term is
// formed before the scatter from global loads of x and its neighbours.
template <class TO, bool D3, int NN, int MINW, bool ROW>
__global__ __launch_bounds__(NN * 4, MINW) void apply_mfma_kernel(Slots sl, const float* __restrict__ x,
                                                             TO* __restrict__ y, const float* __restrict__ sT,
                                                             const float* __restrict__ sA,
                                                             const float* __restrict__ S,
                                                             const float* __restrict__ dc,
                                                             const int* __restrict__ sg, int nx, int ny, int nz,
                                                             int cells) {
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  x = at(x, bs.ws + bs.dx);
  y = at(y, bs.ws + bs.dy);
  sT = at(sT, bs.op);
  sA = at(sA, bs.op);
  S = at(S, bs.op);
  dc = at(dc, bs.op);
  sg = at(sg, bs.op);
  constexpr int KS = NN / 32;       // k-steps of the MFMA (32 directions each)
  constexpr int NT = NN * 4;        // threads: NN / 16 waves
  constexpr int LDR = NN + 8;       // plane row: the directions of one cell, padded
  constexpr int NA = D3 ? 3 : 2;
  constexpr int XR = 68;             // FP32 tile row: one direction, halo at 3 and 68
  __shared__ uint16_t xp[3][64 * LDR];
  __shared__ float xf[ROW ? NN * XR + 4 : 1];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int li = lane & 15, grp = lane >> 4;
  const int ntile = cells / 64;
  const int G = int(gridDim.x);
  int t0, tstep, tend;
  if ((ntile & 7) == 0 && (G & 7) == 0) {
    const int k = int(blockIdx.x) & 7;
    t0 = k * (ntile >> 3) + (int(blockIdx.x) >> 3);
    tstep = G >> 3;
    tend = (k + 1) * (ntile >> 3);
  } else {
    t0 = int(blockIdx.x);
    tstep = G;
    tend = ntile;
  }
  if (t0 >= tend) return;

  // split of one value into three bfloat16 terms
  auto split3 = [](float v, uint16_t& h0, uint16_t& h1, uint16_t& h2) {
    const __bf16 b0 = __bf16(v);
    const float r1 = v - float(b0);
    const __bf16 b1 = __bf16(r1);
    const float r2 = r1 - float(b1);
    const __bf16 b2 = __bf16(r2);
    h0 = __builtin_bit_cast(uint16_t, b0);
    h1 = __builtin_bit_cast(uint16_t, b1);
    h2 = __builtin_bit_cast(uint16_t, b2);
  };
  // the same split of two values at once, each term a packed pair (first
  // value in the low half): one conversion per term and pair
  auto split3x2 = [](float a, float b, uint32_t& p0, uint32_t& p1, uint32_t& p2) {
    p0 = __builtin_bit_cast(uint32_t, __builtin_convertvector(v2f{a, b}, v2bf));
    const float a1 = a - __uint_as_float(p0 << 16), b1 = b - __uint_as_float(p0 & 0xffff0000u);
    p1 = __builtin_bit_cast(uint32_t, __builtin_convertvector(v2f{a1, b1}, v2bf));
    const float a2 = a1 - __uint_as_float(p1 << 16), b2 = b1 - __uint_as_float(p1 & 0xffff0000u);
    p2 = __builtin_bit_cast(uint32_t, __builtin_convertvector(v2f{a2, b2}, v2bf));
  };
  // the wave's rows of S as A operands: lane l holds S[16 w + l % 16][32 ks + 8 (l / 16) + e]
  v8bf sa[3][KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const float* __restrict__ srow = S + (16 * wave + li) * NN + 32 * ks + 8 * grp;
    uint16_t h[3][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) split3(srow[e], h[0][e], h[1][e], h[2][e]);
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int e = 0; e < 8; ++e) sa[p][ks][e] = __builtin_bit_cast(__bf16, h[p][e]);
  }
  float dcv[4][NA];
  int sgv[4][NA];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const int m = 16 * wave + 4 * grp + r;
      dcv[r][a] = dc[4 * m + a];
      sgv[r][a] = sg[4 * m + a];
    }
  const int ext[3] = {nx, ny, nz};
  const int stride[3] = {1, nx, nx * ny};
  int64_t rowb[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) rowb[r] = int64_t(16 * wave + 4 * grp + r) * cells;

  // staging: thread (g, q) takes directions 4 g .. 4 g + 3 of cells 4 q .. 4 q + 3;
  // each 16-lane group takes two consecutive direction quads g and eight cell
  // quads q, so its loads are two whole 128-byte rows and its 8-byte plane
  // stores fall on distinct banks (with the row order below)
  const int tk = int(threadIdx.x) >> 4;
  const int sg4 = 2 * (tk >> 1) + ((int(threadIdx.x) >> 3) & 1);
  const int sq = (int(threadIdx.x) & 7) + 8 * (tk & 1);
  // plane row of tile cell c: bits 0-1 of c XOR bits 2-3, bits 2-3 XOR bits
  // 4-5.  Rows of 16 B-fragment reads (16 consecutive cells) and of staging
  // stores (cells 4 q + j over the group's q) then cover every bank equally
  auto prow = [](int c) { return c ^ ((c >> 2) & 3) ^ (((c >> 4) & 3) << 2); };
  int rrow[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) rrow[u] = prow(16 * u + li) * LDR;
  // (S x)^T for the wave's directions at the tile's 64 cells, from the planes:
  // per k-step and x term (x2, x1, x0) its fragments are read once from LDS,
  // then its products with S0 .. S(2 - term), so the six products run
  // smallest first; u innermost so that consecutive MFMAs do not wait on
  // each other's results
  auto scatter = [&](v4f(&acc)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int p = 2; p >= 0; --p) {
        v8bf bx[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          bx[u] = *reinterpret_cast<const v8bf*>(&xp[p][rrow[u] + 32 * ks + 8 * grp]);
#pragma unroll
        for (int q = 2 - p; q >= 0; --q)
#pragma unroll
          for (int u = 0; u < 4; ++u)
            acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sa[q][ks], bx[u], acc[u], 0, 0, 0);
      }
  };
  v4f rx[4];
  auto load_x = [&](int tile) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      rx[i] = *reinterpret_cast<const v4f*>(x + int64_t(4 * sg4 + i) * cells + tile * 64 + 4 * sq);
  };
  // whole-row tiles (64 | nx): the block also keeps the tile in FP32, one
  // row per direction with the x-neighbours of its end cells as halo (zero
  // outside the domain), so x at the lane's cells and its upwind x-neighbour
  // come from LDS; the y / z neighbours are loads at byte offsets fixed per
  // lane (own cell, or the upwind one) from the tile's first cell
  float hv = 0.f;  // the halo value of this thread (threads 0 .. 2N - 1)
  auto load_halo = [&](int tile) {
    if (int(threadIdx.x) < 2 * NN) {
      const int d = int(threadIdx.x) >> 1, right = int(threadIdx.x) & 1;
      const int c0 = tile * 64, ti = c0 % nx;
      const bool in = right ? ti + 64 < nx : ti > 0;
      const float v = x[int64_t(d) * cells + (in ? (right ? c0 + 64 : c0 - 1) : c0)];
      hv = in ? v : 0.f;
    }
  };
  // per r: LDS index of the lane's cell and of its x-neighbour; byte offsets
  // in x of the lane's cell and of its upwind neighbours, less the tile's
  // first cell's, taken modulo 2^32 (the host sends only vectors of fewer
  // than 2^30 elements here, so adding the tile's own offset gives the exact
  // offset of any cell inside the domain)
  int xb[4], xn[4];
  uint32_t ob[4], qb[4][NA];
  float dsum[4];              // sum over axes of the upwind coefficients
  if constexpr (ROW) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 16 * wave + 4 * grp + r;
      xb[r] = m * XR + 4 + li;
      xn[r] = xb[r] - sgv[r][0];
      ob[r] = uint32_t(rowb[r] + li) * uint32_t(sizeof(float));
      dsum[r] = 0.f;
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        qb[r][a] = ob[r] - uint32_t(sgv[r][a] * stride[a]) * uint32_t(sizeof(float));
        dsum[r] += dcv[r][a];
      }
    }
    load_halo(t0);
  }
  load_x(t0);
  for (int tile = t0; tile < tend; tile += tstep) {
    const int c0 = tile * 64;
    if (tile != t0) __syncthreads();  // the previous tile's reads of the planes are done
    if constexpr (ROW) {
#pragma unroll
      for (int i = 0; i < 4; ++i) *reinterpret_cast<v4f*>(&xf[(4 * sg4 + i) * XR + 4 + 4 * sq]) = rx[i];
      if (int(threadIdx.x) < 2 * NN)
        xf[(int(threadIdx.x) >> 1) * XR + ((threadIdx.x & 1) ? XR : 3)] = hv;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {  // cell 4 sq + j: four directions per plane, 8 bytes each
      uint32_t lo[3], hi[3];
      split3x2(rx[0][j], rx[1][j], lo[0], lo[1], lo[2]);
      split3x2(rx[2][j], rx[3][j], hi[0], hi[1], hi[2]);
#pragma unroll
      for (int p = 0; p < 3; ++p)
        *reinterpret_cast<v2u*>(&xp[p][prow(4 * sq + j) * LDR + 4 * sg4]) = v2u{lo[p], hi[p]};
    }
    if constexpr (!ROW) {
      // the streaming term and x at the lane's cells, formed before the
      // scatter so that the neighbours' registers are free during it
      float st[4], sav[4], xcv[4][4], str[4][4];
      int ti0 = 0, tj = 0, tk = 0;
      if ((nx & 63) == 0) {
        const int rr = c0 / nx;
        ti0 = c0 - rr * nx;
        tj = rr % ny;
        tk = rr / ny;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + 16 * u + li;
        st[u] = sT[c];
        sav[u] = sA[c];
        int pos[3];
        if ((nx & 63) == 0) {
          pos[0] = ti0 + 16 * u + li;
          pos[1] = tj;
          pos[2] = tk;
        } else {
          const int rr = c / nx;
          pos[0] = c - rr * nx;
          pos[1] = rr % ny;
          pos[2] = rr / ny;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t o = rowb[r] + c;
          float nb[NA];
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            const int pp = pos[a] - sgv[r][a];
            const bool inb = unsigned(pp) < unsigned(ext[a]);
            const float v = x[inb ? o - sgv[r][a] * stride[a] : o];
            nb[a] = inb ? v : 0.f;
          }
          const float xc = x[o];
          float sr = 0.f;
#pragma unroll
          for (int a = 0; a < NA; ++a) sr += dcv[r][a] * (xc - nb[a]);
          xcv[u][r] = xc;
          str[u][r] = sr;
        }
      }
      if (tile + tstep < tend) load_x(tile + tstep);  // in flight during this tile's work
      __syncthreads();
      v4f acc[4];
      scatter(acc);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + 16 * u + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float xc = xcv[u][r], sx = acc[u][r];
          y[rowb[r] + c] = TO(str[u][r] + st[u] * (xc - sx) + sav[u] * sx);
        }
      }
    } else {
      // the y / z neighbours (the lane's own cell where the upwind one is
      // outside the domain, its coefficient then taken as zero) and the
      // cross sections, requested before the scatter
      const int rr = c0 / nx, tj = rr % ny, tk = rr / ny;
      const int pos[3] = {0, tj, tk};
      const char* __restrict__ xc8 = reinterpret_cast<const char*>(x);
      const uint32_t tb = uint32_t(c0) * uint32_t(sizeof(float));
      float dcm[4][NA], nb[4][4][NA];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int a = 1; a < NA; ++a) {
          const bool inb = unsigned(pos[a] - sgv[r][a]) < unsigned(ext[a]);
          dcm[r][a] = inb ? dcv[r][a] : 0.f;
          const uint32_t off = tb + (inb ? qb[r][a] : ob[r]);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            nb[u][r][a] = *reinterpret_cast<const float*>(xc8 + off + 64 * u);
        }
      float st[4], sav[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        st[u] = sT[c0 + 16 * u + li];
        sav[u] = sA[c0 + 16 * u + li];
      }
      if (tile + tstep < tend) {  // in flight during this tile's work
        load_x(tile + tstep);
        load_halo(tile + tstep);
      }
      __syncthreads();
      v4f acc[4];
      scatter(acc);
      // x and the x-neighbour from LDS; the streaming term as x times the
      // summed coefficients less each coefficient times its neighbour (zero
      // outside the domain), then the collision and scatter terms
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t yo = uint32_t(c0) + (ob[r] >> 2);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float xc = xf[xb[r] + 16 * u], sx = acc[u][r];
          float sr = xc * dsum[r] - dcv[r][0] * xf[xn[r] + 16 * u];
#pragma unroll
          for (int a = 1; a < NA; ++a) sr -= dcm[r][a] * nb[u][r][a];
          y[yo + uint32_t(16 * u)] = TO(sr + st[u] * (xc - sx) + sav[u] * sx);
        }
      }
    }
  }
}

// FP64 apply and residual (y = L x or y = b - L x, FP64 throughout) with
// the scatter on the FP64 matrix cores: for 16 cells, (S x)[m] over all N
// directions is an [N x N] by [N x 16] product, 16x16 output tiles with
// k-groups of 4 (mfma_f64_16x16x4f64: lane l supplies row l mod 16 of A and
// column l mod 16 of B for k-group l / 16; its i-th result is D row
// l / 16 + 4 i of column l mod 16, interleaved unlike the FP32 16x16x4 form,
// as measured on gfx950).  A is S, held in LDS in fragment order (the 64 values
// of one tile and k-group in lane order: one conflict-free read per MFMA); B
// is x, each lane loading its cell's values of directions 4 ks + l / 16
// straight from global memory, 128 contiguous bytes per k-group row, once per
// 16 cells for all N / 16 direction tiles.  The D rows are four directions of
// one cell per lane, so the epilogue (upwind streaming, collision, b) reads
// and writes 128-byte row segments too.  A wave takes one 16-cell tile at a
// time; a block's four waves walk a contiguous range of tiles (neighbouring
// rows stay in one L2).  The epilogue operands of a pass's direction tiles
// are requested before its MFMAs; the per-direction upwind signs and
// coefficients sit in LDS beside S, so that no neighbour address waits on a
// global load (that took the 512^2 x 64 residual from 190 to 120 us).  The FP64
// MFMA accumulates its four products per k-group in order, as the vector
// kernel's fused multiply-adds do: the two agree bit for bit (measured).
typedef double v4d __attribute__((ext_vector_type(4)));

// The register budget (three waves per SIMD up to 64 directions) changes no
// timing; left to itself the compiler took about 190 VGPRs for epilogue
// loads in flight.
template <bool RES, bool D3, int NN>
__global__ __launch_bounds__(256, NN <= 64 ? 3 : 2) void apply64_mfma_kernel(Slots sl, const double* __restrict__ x,
                                                           double* __restrict__ y, const double* __restrict__ b,
                                                           const double* __restrict__ sT,
                                                           const double* __restrict__ sA,
                                                           const double* __restrict__ S,
                                                           const double* __restrict__ dc,
                                                           const int* __restrict__ sg, int nx, int ny, int nz,
                                                           int cells, int per_block) {
  static_assert(NN % 16 == 0, "direction tiles of 16");
  constexpr int KS = NN / 4;   // k-groups
  constexpr int MT = NN / 16;  // direction tiles
  // direction tiles per pass: two independent MFMA chains at 96 directions;
  // one at 64 and below (fewer registers; measured residuals: 120 against
  // 125 us at 512^2 x 64, 231 against 228 us at 64^3 x 96)
  constexpr int MP = NN == 96 ? 2 : 1;
  SlotBase bs;
  if (!slot_open(sl, blockIdx.z, bs)) return;
  x = at(x, bs.ws + bs.dx);
  y = at(y, bs.ws + bs.dy);
  if (RES) b = at(b, bs.ws);
  sT = at(sT, bs.op);
  sA = at(sA, bs.op);
  S = at(S, bs.op);
  dc = at(dc, bs.op);
  sg = at(sg, bs.op);
  constexpr int NA = D3 ? 3 : 2;
  __shared__ double Sf[NN * NN];
  // per direction and axis: the streaming coefficient and the upwind
  // neighbour's signed offset in cells (LDS, so that no neighbour address
  // waits on a global load)
  __shared__ double dcs[NN * NA];
  __shared__ int sgs[NN * NA];
  for (int idx = threadIdx.x; idx < NN * NN; idx += 256) {
    const int l = idx & 63, f = idx >> 6;
    const int mt = f / KS, ks = f - (f / KS) * KS;
    Sf[idx] = S[(mt * 16 + (l & 15)) * NN + ks * 4 + (l >> 4)];
  }
  for (int idx = threadIdx.x; idx < NN * NA; idx += 256) {  // 288 entries at 96 directions in 3D
    const int m = idx / NA, a = idx - (idx / NA) * NA;
    dcs[idx] = dc[4 * m + a];
    sgs[idx] = sg[4 * m + a];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const int li = lane & 15, grp = lane >> 4;
  const int ntile = (cells + 15) >> 4;
  const int g = int(gridDim.x);
  const int t0 = xcd_tile(int(blockIdx.x), g) * per_block;
  const int t1 = t0 + per_block < ntile ? t0 + per_block : ntile;
  const int stride[3] = {1, nx, nx * ny};
  const int ext[3] = {nx, ny, nz};
  // element offsets as 32-bit byte offsets from the vector's base (the host
  // guarantees 8 n < 2^32): one VGPR per address
  const char* __restrict__ x8 = reinterpret_cast<const char*>(x);
  const char* __restrict__ b8 = reinterpret_cast<const char*>(b);
  char* __restrict__ y8 = reinterpret_cast<char*>(y);
  auto ld = [](const char* base, uint32_t off) { return *reinterpret_cast<const double*>(base + off); };
  const uint32_t row8 = uint32_t(cells) * 8u;
  for (int t = t0 + wave; t < t1; t += 4) {
    const int c = t * 16 + li;
    const bool live = c < cells;
    const int cc = live ? c : cells - 1;  // past the end: compute on the last cell, store nothing
    const uint32_t cb = uint32_t(cc) * 8u;
    double xb[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) xb[ks] = ld(x8, uint32_t(ks * 4 + grp) * row8 + cb);
    const int rr = cc / nx;
    const int pos[3] = {cc - rr * nx, rr - (rr / ny) * ny, rr / ny};
    const double st = sT[cc], sa = sA[cc];
#pragma unroll 1
    for (int mt0 = 0; mt0 < MT; mt0 += MP) {
      // epilogue operands of the pass's directions, requested first
      double xc[MP][4], str[MP][4], bv[MP][4];
#pragma unroll
      for (int p = 0; p < MP; ++p)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = (mt0 + p) * 16 + grp + 4 * i;
          const uint32_t o = uint32_t(m) * row8 + cb;
          const double v = ld(x8, o);
          double sacc = 0.0;
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            const int sgn = sgs[m * NA + a];
            const int q = pos[a] - sgn;
            const bool inb = q >= 0 && q < ext[a];
            const double nb = ld(x8, inb ? o - uint32_t(sgn * stride[a]) * 8u : o);
            sacc += dcs[m * NA + a] * (v - (inb ? nb : 0.0));
          }
          xc[p][i] = v;
          str[p][i] = sacc;
          bv[p][i] = RES ? ld(b8, o) : 0.0;
        }
      v4d acc[MP];
#pragma unroll
      for (int p = 0; p < MP; ++p) acc[p] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int p = 0; p < MP; ++p)
          acc[p] = __builtin_amdgcn_mfma_f64_16x16x4f64(Sf[((mt0 + p) * KS + ks) * 64 + lane], xb[ks], acc[p],
                                                        0, 0, 0);
      if (live) {
#pragma unroll
        for (int p = 0; p < MP; ++p)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int m = (mt0 + p) * 16 + grp + 4 * i;
            const double val = str[p][i] + st * (xc[p][i] - acc[p][i]) + sa * acc[p][i];
            *reinterpret_cast<double*>(y8 + (uint32_t(m) * row8 + cb)) = RES ? bv[p][i] - val : val;
          }
      }
    }
  }
}

// FP64 apply / residual on the matrix cores for 16, 32, 64 or 96 directions;
// false for other counts (the vector kernel takes them)
template <bool RES>
bool go_mfma64(const Target& Tg, const void* x, void* y, const double* b, hipStream_t s, const ProfScope& ps) {
  const Operator& op = *Tg.op;
  const OpArrays& A = Tg.arr;
  const int N = op.ndir;
  if (N != 16 && N != 32 && N != 64 && N != 96) return false;
  if (op.n >= (int64_t(1) << 29)) return false;  // byte offsets of one vector in 32 bits
  const int ntile = int((op.cells + 15) / 16);
  // blocks over all solves of the launch, about as many as the CUs hold at
  // once, each a contiguous range of 16-cell tiles of one solve (whole
  // 4-tile rounds); a multiple of 8 when the grid is split (XCD order)
  const int rounds = (ntile + 3) / 4;
  // 1024 blocks in all: a sweep of 256 to 8192 at 512^2 x 64 and 64^3 x 96
  // directions gave 121 and 233 us at 1024, 124 to 175 and 243 to 287 us
  // otherwise; a walk of each block's tiles down a column of row segments
  // (so that the upwind rows are sibling waves' tiles) measured no faster
  int64_t g = std::max<int64_t>(1, 1024 / std::max(1, Tg.sl.count));
  g = std::min<int64_t>(g, rounds);
  if (g >= 8) g &= ~int64_t(7);
  const int per_block = int(4 * ((rounds + g - 1) / g));
  const dim3 grid(unsigned(g), 1, unsigned(Tg.sl.count));
  const bool d3 = op.nz > 1;
  auto launch = [&](auto kern) {
    launch_k(kern, grid, dim3(256), 0u, s, ps, Tg.sl, static_cast<const double*>(x), static_cast<double*>(y), b,
             A.sT64, A.sA64, A.S64, A.dc64, static_cast<const int*>(A.dsgn), op.nx, op.ny, op.nz, int(op.cells),
             per_block);
  };
  switch (N) {
    case 16: d3 ? launch(apply64_mfma_kernel<RES, true, 16>) : launch(apply64_mfma_kernel<RES, false, 16>); break;
    case 32: d3 ? launch(apply64_mfma_kernel<RES, true, 32>) : launch(apply64_mfma_kernel<RES, false, 32>); break;
    case 64: d3 ? launch(apply64_mfma_kernel<RES, true, 64>) : launch(apply64_mfma_kernel<RES, false, 64>); break;
    default: d3 ? launch(apply64_mfma_kernel<RES, true, 96>) : launch(apply64_mfma_kernel<RES, false, 96>); break;
  }
  return true;
}

template <class TO, bool D3>
bool go_mfma(const Target& Tg, const void* x, void* y, hipStream_t s, const ProfScope& ps) {
  const Operator& op = *Tg.op;
  const OpArrays& A = Tg.arr;
  if (op.cells % 64 != 0) return false;
  // whole-row tiles: 64 divides nx and byte offsets of x fit in 32 bits
  const bool row = op.nx % 64 == 0 && op.n < (int64_t(1) << 30);
  // blocks over all solves of the launch: as many as the CUs hold at once
  // (three per CU in 2D, whose register budget gives three waves per SIMD;
  // 512 in 3D), each walking several tiles of a single solve, at least one
  // tile each; a multiple of 8 when the tile count is (the XCD-contiguous
  // order).  Measured with whole-row tiles at 512^2 x 64 and 64^3 x 96
  // directions: 512 blocks 33.3 and 67.0 us, 768 30.8 and 74.7 us; before
  // (every neighbour a global load) 512 blocks 48.5 and 119 us, 1024 50.6
  // and 132 us, 2048 52.1 and 147 us, 4096 63.8 and 178 us, 256 60.7 and
  // 117 us.  Staging the upwind y/z neighbours as whole coalesced tile
  // segments in LDS (instead of per-lane loads) measured no faster.
  const int64_t ntile = op.cells / 64;
  const int base = (D3 ? 512 : 768) * (op.ndir == 32 ? 2 : 1);  // 32 directions: two-wave blocks
  int64_t g = std::max<int64_t>(1, base / std::max(1, Tg.sl.count));
  if (ntile % 8 == 0) g = std::max<int64_t>(8, g & ~int64_t(7));
  g = std::min(g, ntile);
  const dim3 grid(unsigned(g), 1, unsigned(Tg.sl.count));
  auto launch = [&](auto kern, int nn) {
    launch_k(kern, grid, dim3(unsigned(4 * nn)), 0u, s, ps, Tg.sl, static_cast<const float*>(x),
             static_cast<TO*>(y), A.sT32, A.sA32, A.S32, A.dc32, static_cast<const int*>(A.dsgn), op.nx, op.ny,
             op.nz, int(op.cells));
  };
  // 32, 64 and 96 directions.  At 32 (two-wave blocks, twice as many): a
  // single 256^2 apply 7.9 us against 10.3 us on the vector kernel, 64^2 and
  // 128^2 equal (8 us, launch-bound); the serving stream's throughput is
  // unchanged (measured)
  // waves per SIMD the register budget is cut to: three in 2D (no spills);
  // two in 3D, whose three upwind neighbours per value would spill at three
  // (measured at 64^3 x 96: 95 us at two, 114 us at three)
  constexpr int MW = D3 ? 2 : 3;
  switch (op.ndir) {
    case 32:
      row ? launch(apply_mfma_kernel<TO, D3, 32, MW, true>, 32) : launch(apply_mfma_kernel<TO, D3, 32, MW, false>, 32);
      return true;
    case 64:
      row ? launch(apply_mfma_kernel<TO, D3, 64, MW, true>, 64) : launch(apply_mfma_kernel<TO, D3, 64, MW, false>, 64);
      return true;
    case 96:
      row ? launch(apply_mfma_kernel<TO, D3, 96, MW, true>, 96) : launch(apply_mfma_kernel<TO, D3, 96, MW, false>, 96);
      return true;
    default: return false;
  }
}

template <class T, class TI, class TO, bool RES, bool LDS_S, int TL>
void go_dpt(const Target& Tg, const void* x, void* y, const double* b, const T* sT, const T* sA, const T* S,
            const T* dc, size_t lds, hipStream_t s, const ProfScope& ps) {
  const Operator& op = *Tg.op;
  // FP64: 512 threads, so each thread carries half the directions (at 64
  // directions 16 per thread took 260 VGPRs and one wave per SIMD)
  constexpr int NT = sizeof(T) == 8 ? 512 : 256;
  constexpr int DSLOTS = NT / TL;
  const dim3 grid(unsigned((op.cells + TL - 1) / TL), 1, unsigned(Tg.sl.count));
  const int dpt = (op.ndir + DSLOTS - 1) / DSLOTS;
  auto launch = [&](auto kern) {
    launch_k(kern, grid, dim3(NT), uint32_t(lds), s, ps, Tg.sl, static_cast<const TI*>(x), static_cast<TO*>(y),
             b, sT, sA, S, dc, static_cast<const int*>(Tg.arr.dsgn), op.ndir, op.nx, op.ny, op.nz,
             int(op.cells));
  };
  if (dpt <= 1)
    launch(apply_kernel<T, TI, TO, RES, LDS_S, 1, TL, NT>);
  else if (dpt <= 2)
    launch(apply_kernel<T, TI, TO, RES, LDS_S, 2, TL, NT>);
  else if (dpt <= 4)
    launch(apply_kernel<T, TI, TO, RES, LDS_S, 4, TL, NT>);
  else if (dpt <= 8)
    launch(apply_kernel<T, TI, TO, RES, LDS_S, 8, TL, NT>);
  else if constexpr (NT == 256)  // with 512 threads at most 256 / 32 directions per thread
    launch(apply_kernel<T, TI, TO, RES, LDS_S, 16, TL, NT>);
  else
    throw Error(RTE_EINVAL, "apply: more directions per thread than the launch supports");
}

template <class T, class TI, class TO, bool RES>
void go(const Target& Tg, const void* x, void* y, const double* b, hipStream_t s, const ProfScope& ps) {
  const OpArrays& A = Tg.arr;
  const T* sT;
  const T* sA;
  const T* S;
  const T* dc;
  if constexpr (sizeof(T) == 8) {
    sT = A.sT64; sA = A.sA64; S = A.S64; dc = A.dc64;
  } else {
    sT = A.sT32; sA = A.sA32; S = A.S32; dc = A.dc32;
  }
  const int N = Tg.op->ndir;
  const bool wide = N <= 64;
  const int tl = wide ? 64 : 16;
  const size_t lx = size_t(N) * tl * sizeof(T);
  const size_t ls = size_t(N) * size_t(wide ? N : N + 1) * sizeof(T);
  const bool lds_s = lx + ls <= size_t(kApplyLds);
  // without S in LDS the 16-cell tiles stage S in chunks of columns
  const size_t lds =
      lds_s ? lx + ls : (wide ? lx : lx + size_t(N) * size_t(apply_s_chunk(N, tl, int(sizeof(T))) + 1) * sizeof(T));
  if (wide) {
    if (lds_s)
      go_dpt<T, TI, TO, RES, true, 64>(Tg, x, y, b, sT, sA, S, dc, lds, s, ps);
    else
      go_dpt<T, TI, TO, RES, false, 64>(Tg, x, y, b, sT, sA, S, dc, lds, s, ps);
  } else {
    if (lds_s)
      go_dpt<T, TI, TO, RES, true, 16>(Tg, x, y, b, sT, sA, S, dc, lds, s, ps);
    else
      go_dpt<T, TI, TO, RES, false, 16>(Tg, x, y, b, sT, sA, S, dc, lds, s, ps);
  }
  RTE_HIP(hipGetLastError());
}

// RTE_APPLY64_VEC=1 keeps the FP64 apply and residual on the vector kernel
// (for comparisons)
bool mfma64_off() {
  const char* e = std::getenv("RTE_APPLY64_VEC");
  return e && e[0] == '1';
}

}  // namespace

void launch_apply(const Target& Tg, const void* x, int tin, void* y, int tout, const double* b, bool fp64,
                  hipStream_t s) {
  const Operator& op = *Tg.op;
  const double unknowns = double(op.n), cells = double(op.cells);
  if (b) {
    RTE_REQUIRE(fp64 && tin == 1 && tout == 1, RTE_EINVAL, "residual is FP64 only");
    ProfScope ps(RTE_K_RESIDUAL, s, true);
    ps.work = 24.0 * unknowns + 16.0 * cells;  // x, b in; r out; sT, sA
    if (!mfma64_off() && go_mfma64<true>(Tg, x, y, b, s, ps)) return;
    go<double, double, double, true>(Tg, x, y, b, s, ps);
    return;
  }
  ProfScope ps(RTE_K_APPLY, s, true);
  const double esz[2] = {4.0, 8.0};
  ps.work = (esz[tin] + esz[tout]) * unknowns + (fp64 ? 16.0 : 8.0) * cells;
  if (fp64) {
    RTE_REQUIRE(tin == 1 && tout == 1, RTE_EINVAL, "FP64 apply takes FP64 vectors");
    if (mfma64_off() || !go_mfma64<false>(Tg, x, y, nullptr, s, ps)) go<double, double, double, false>(Tg, x, y, nullptr, s, ps);
  } else if (tin == 0 && (op.nz > 1 ? (tout == 0 ? go_mfma<float, true>(Tg, x, y, s, ps)
                                                  : go_mfma<double, true>(Tg, x, y, s, ps))
                                     : (tout == 0 ? go_mfma<float, false>(Tg, x, y, s, ps)
                                                  : go_mfma<double, false>(Tg, x, y, s, ps)))) {
    // the matrix-core scatter (N of 32, 64 or 96, whole 64-cell tiles)
  } else if (tin == 0 && Tg.arr.Sp32 && slot_budget(op.ndir) > 0) {
    const bool d3 = op.nz > 1;
    if (tout == 0)
      d3 ? go_slot<float, true>(Tg, x, y, s, ps) : go_slot<float, false>(Tg, x, y, s, ps);
    else
      d3 ? go_slot<double, true>(Tg, x, y, s, ps) : go_slot<double, false>(Tg, x, y, s, ps);
  } else if (tin == 0 && tout == 0) {
    go<float, float, float, false>(Tg, x, y, nullptr, s, ps);
  } else if (tin == 0 && tout == 1) {
    go<float, float, double, false>(Tg, x, y, nullptr, s, ps);
  } else {
    go<float, double, float, false>(Tg, x, y, nullptr, s, ps);
  }
}

}  // namespace rte

// Internal declarations shared by the librte sources (not part of the ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/rte.h"

namespace rte {

// ---------------------------------------------------------------- errors ---
struct Error : std::runtime_error {
  rte_status code;
  Error(rte_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};
[[noreturn]] void fail(rte_status code, const std::string& msg);
void set_last_error(const std::string& msg);

#define RTE_HIP(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      ::rte::fail(RTE_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
  } while (0)

#define RTE_REQUIRE(cond, code, msg)        \
  do {                                      \
    if (!(cond)) ::rte::fail((code), (msg)); \
  } while (0)

// Device allocations owned by a handle; freed on destruction.
struct DevArena {
  std::vector<void*> ptrs;
  template <class T>
  T* alloc(size_t count) {
    void* p = nullptr;
    size_t bytes = count * sizeof(T);
    if (bytes == 0) bytes = 256;
    RTE_HIP(hipMalloc(&p, bytes));
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  template <class T>
  T* upload(const std::vector<T>& host) {
    T* d = alloc<T>(host.size());
    if (!host.empty()) RTE_HIP(hipMemcpy(d, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
  }
  ~DevArena() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

uint16_t bf16_rne(float f);

// ----------------------------------------------------- batched launches ---
// A group of solves of one shape advances together: grid z of every launch
// runs over the group's slots, and each per-solve array argument is an
// offset from the slot's workspace base or operator-block base, both read
// from the slot table.  With no table a launch covers one solve and its
// array arguments are absolute addresses.
//
// Every slot runs its own restart cycle: jj is the slot's Arnoldi step
// within its cycle, so one launch can advance slots that sit at different
// steps.  A cycle ends on the device (the step kernel clears live and sets
// edge); the next boundary launches, gated on edge, form the true residual
// and take the restart-or-finish decision on the device as well.  The host
// only admits solves, launches boundaries and copies finished results out.
struct SlotDesc {
  uint64_t ws;        // workspace base of the solve held by the slot
  uint64_t op;        // operator-block base of that solve
  int32_t live;       // 1 while the solve takes Arnoldi steps
  int32_t occupied;   // 1 while the slot holds a solve
  int32_t jj;         // Arnoldi steps taken in the current cycle
  int32_t limit;      // Arnoldi steps allowed in the current cycle
  double rtol;        // stop the cycle once |g_{j+1}| / ||b|| <= rtol
  int32_t bad;        // a non-finite value appeared in the current cycle
  int32_t edge;       // at a cycle boundary (ended cycle, or a new solve)
  int32_t iters;      // Arnoldi steps of the completed cycles
  int32_t max_iters;  // the solve's iteration limit
  int32_t restarts;   // completed cycles with at least one step
  int32_t stall;      // consecutive boundaries that cut the residual by < 0.1 %
  int32_t done;       // 0 running; 1 finished; 2 finished with x = 0 (b = 0)
  int32_t code;       // rte_status of a finished solve
  int32_t steps;      // Arnoldi steps taken, discarded cycles included
  int32_t pad;
  double bnorm;       // ||b||, negative until the first boundary
  double prev;        // true residual norm at the previous boundary
  double rel;         // true relative residual at the last boundary
};
static_assert(sizeof(SlotDesc) == 104, "slot descriptor layout");

// Work the host stages per slot for one tick and hands over in a single
// transfer and launch: admissions (the descriptor, x0 or null for x = 0, and
// the right-hand side, as absolute device addresses) and finished results
// (copy x to out, or zeros for b = 0).
struct SlotInit {
  SlotDesc d;
  uint64_t x0, b;
  int32_t admit, pad;
};
struct SlotEmit {
  uint64_t out, x;
  int32_t mode, pad;  // 0: nothing, 1: copy x, 2: zeros
};
// For every slot with init[z].admit: x = x0 (or 0) and b copied into the
// workspace at init[z].d.ws + off_x / off_b, then tab[z] = init[z].d.
void launch_admit(SlotDesc* tab, const SlotInit* init, int count, int64_t n, uint64_t off_x, uint64_t off_b,
                  hipStream_t s);
void launch_emit(const SlotEmit* em, int count, int64_t n, hipStream_t s);

// Launch-wide slot selection.  gate picks the slots a launch runs for;
// jx and jy are the bytes one Arnoldi step index adds to a launch's
// step-indexed input and output operand (V_j, Z_j, V_{j+1}), applied with
// the slot's own jj.
enum SlotGate { GATE_LIVE = 0, GATE_OCCUPIED = 1, GATE_EDGE = 2 };
struct Slots {
  SlotDesc* tab = nullptr;
  int count = 1;  // slots covered by the launch (grid z extent)
  int gate = GATE_LIVE;
  int64_t jx = 0, jy = 0;
};

struct SlotBase {
  uint64_t ws = 0, op = 0;
  uint64_t dx = 0, dy = 0;  // step-indexed operand offsets (bytes)
  int jj = 0;
};

// Reads slot z's bases; false when the slot sits this launch out.
__device__ inline bool slot_open(const Slots& sl, int z, SlotBase& b) {
  if (!sl.tab) return true;
  const SlotDesc* d = sl.tab + z;
  b.ws = d->ws;
  b.op = d->op;
  b.jj = d->jj;
  b.dx = uint64_t(int64_t(b.jj) * sl.jx);
  b.dy = uint64_t(int64_t(b.jj) * sl.jy);
  const int open = sl.gate == GATE_LIVE ? d->live : sl.gate == GATE_OCCUPIED ? d->occupied : d->edge;
  return open != 0;
}

// p + base (bytes).  On the device the sum is formed by byte-pointer
// arithmetic on the kernel argument, so the compiler still knows the
// result points to global memory (and keeps global, not flat, loads).
template <class T>
__host__ __device__ inline T* at(T* p, uint64_t base) {
#if defined(__HIP_DEVICE_COMPILE__)
  using C = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return reinterpret_cast<T*>(reinterpret_cast<C*>(p) + base);
#else
  return reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) + base);
#endif
}

// ------------------------------------------------------------ the model ---
// A convolution in GEMM layout: w[tap][cout][cin] (input channels fastest).
struct ConvW {
  int taps = 0, cout = 0, cin = 0;
  std::vector<float> f32;
  std::vector<uint16_t> b16;
  const float* d32 = nullptr;
  const uint16_t* d16 = nullptr;
};

// Per-class tap table of a stride-2 transposed convolution (kernel 4,
// padding 1): for output parity class p, the taps feeding it and the input
// offsets relative to the coarse index.
struct Model {
  int dim = 0, ndir = 0, c0 = 0, levels = 0, nu_pre = 0, nu_post = 0, nu_coarse = 0, coef_ch = 0;
  std::vector<float> w_in, w_out;  // [c0][ndir], [ndir][c0]
  float s = 1.f;
  std::vector<ConvW> A, R, Pr;     // Pr: taps ordered [class][tap of class]
  std::vector<std::vector<ConvW>> Bpre, Bpost;
  std::vector<ConvW> Bc;
  // CoeffNet, kept in the blob's layouts: CW [c][cin][3^d], heads [C][c]
  std::vector<std::vector<float>> CW, CB, HAW, HAB, HIW, HIB;

  std::mutex mu;
  int device = -1;
  DevArena* dev = nullptr;
  const float* d_w_in = nullptr;
  const float* d_w_out = nullptr;
  // the 1x1 weights by wave slot: W_in as [4][ndir][c0/4] (entry (s, m, q) =
  // W_in[s + 4q][m]); W_out as [4][c0][slot_budget(ndir)] (entry (s, c, q) =
  // W_out[s + 4q][c], zero past ndir)
  const float* d_w_in_p = nullptr;
  const float* d_w_out_p = nullptr;
  std::vector<const float*> d_CW, d_CB, d_HAW, d_HAB, d_HIW, d_HIB;
  void ensure_on_device();  // uploads once, on the current device
  ~Model();
};

// --------------------------------------------------------- the operator ---
constexpr int MAX_LEVELS = 8;
struct TfpsHost;

// Kernels that give each of a block's four waves one "direction slot" (the
// directions s, s + 4, s + 8, ...) hold ceil(N / 4) values per thread,
// rounded up to a compile-time budget; 0 when N is beyond the largest.
inline int slot_budget(int N) {
  const int need = (N + 3) / 4;
  for (int b : {1, 2, 4, 8, 16, 24, 32})
    if (need <= b) return b;
  return 0;
}

// The operator's device arrays.  They live in one block whose layout
// depends only on the shape (dim, grid, directions, model levels and
// channels), so operators of one shape have them at equal offsets.
struct OpArrays {
  double* b64 = nullptr;      // [n]
  float* sT32 = nullptr;      // sigma_T / eps            [cells]
  float* sA32 = nullptr;      // eps sigma_a              [cells]
  double* sT64 = nullptr;
  double* sA64 = nullptr;
  float* S32 = nullptr;       // [N][N]
  double* S64 = nullptr;
  float* dc32 = nullptr;      // per direction: |u_x|/h, |u_y|/h, |u_z|/h, sum  [N][4]
  double* dc64 = nullptr;
  int* dsgn = nullptr;        // per direction: sign(u_x), sign(u_y), sign(u_z)   [N][4]
  float* Sdiag32 = nullptr;   // S_mm                    [N]
  float* Sp32 = nullptr;      // S by direction slot: [4][N][slot_budget(N)], entry (s, n, q) = S_{s+4q, n}
  float* fa[MAX_LEVELS] = {};     // CoeffNet fields per level [cells_l][C_l]
  float* fainv[MAX_LEVELS] = {};
  // TFPS (Sec. 2.2): per cell the index of its eigen-basis and its particular
  // solution; tf_tab holds the device addresses of the basis tables (kept
  // outside the block so that its layout depends on the shape only):
  // tf_tab[0] -> L^T [nbasis][2N][N] FP64, tf_tab[1] -> xi [nbasis][2N] FP64
  int* tf_bid = nullptr;
  double* tf_chis = nullptr;
  uint64_t* tf_tab = nullptr;
};

struct Operator {
  int dim = 2, nx = 0, ny = 0, nz = 1, ndir = 0, kernel = 0;
  int scheme = RTE_SCHEME_UPWIND;
  int nbasis = 0;                   // TFPS: distinct eigen-bases
  std::shared_ptr<const TfpsHost> tfps_host;  // TFPS: the host build (bases, b), for ATFPS
  int64_t cells = 0, n = 0;
  double h = 0, g = 0;
  int device = 0;
  std::vector<double> S;            // [N][N] host copy
  DevArena mem;
  char* block = nullptr;            // device block holding every array below
  size_t block_bytes = 0;
  OpArrays a;                       // absolute addresses
  const Model* model = nullptr;     // CoeffNet fields were built for this model
  int levels = 0, c0 = 0;           // of that model (0 without one)
  int64_t level_cells(int l) const;
  int level_dim(int l, int axis) const;
  OpArrays relative() const;        // offsets from `block`
  // operators with equal shape keys share the block layout
  std::vector<int64_t> shape_key() const;
  // The geometry of this operator (dimensions, directions, model levels and
  // channels) with no device arrays: what launches need to size themselves,
  // kept by a batch that outlives the operator it was created for.
  std::unique_ptr<Operator> geometry() const;
};

// What a launch addresses: the operator's shape, its arrays (absolute, or
// offsets from each slot's operator block) and the slots it covers.
struct Target {
  const Operator* op;
  OpArrays arr;
  Slots sl;
  static Target single(const Operator& o) { return Target{&o, o.a, Slots{}}; }
};

// ------------------------------------------------------------ launchers ---
struct ApplyGeom {
  int N, nx, ny, nz;
  int64_t cells;
};

// y = L x (res = 0) or y = b - L x (res = 1).  tin/tout: 0 float, 1 double;
// compute precision follows `fp64`.
void launch_apply(const Target& T, const void* x, int tin, void* y, int tout, const double* b, bool fp64,
                  hipStream_t s);
// z = B^{-1} v cell by cell (Block-Jacobi), FP32; v times vscale[0] when given
void launch_block_jacobi(const Target& T, const double* v, const double* vscale, float* z, hipStream_t s);

// MgNet pieces
// STORE_T: out = conv and out2 = a^{-1} (.) conv (a level's first smoothing input)
enum ConvMode { CONV_STORE = 0, CONV_ACCUM = 1, CONV_STORE_T = 2, CONV_RESID_R = 3, CONV_RESID_T = 4 };
enum MfmaKind { MFMA_F32 = 0, MFMA_BF16 = 1 };

struct ConvLaunch {
  Slots sl;
  const float* in;
  int in_dim[3];
  int cin;
  const ConvW* w;
  float* out;
  int out_dim[3];
  int cout;
  int g_dim[3];
  int dim;
  int cstride, ostride;
  int nclass, ntap;
  int8_t obase[8][3];
  int8_t toff[64][3];
  int mode;
  const float* f;
  const float* a;
  const float* ainv;
  float* out2;
  // BF16 path, tiled 2D kernel only: the input is a t tensor stored as
  // bfloat16 (STORE, ACCUM, STORE_T), or the t output -- out of RESID_T and
  // RESID_R, out2 of STORE_T -- is stored as bfloat16
  int in16, t16;
};
void launch_conv(const ConvLaunch& c, int kind, hipStream_t s);
void conv3_setup(ConvLaunch& c, int dim, const int in_dim[3], int stride);
void convT4_setup(ConvLaunch& c, int dim, const int in_dim[3]);

// The operator of either scheme: launch_apply for the upwind one, the TFPS
// apply for the other (same argument meaning).
void launch_operator(const Target& T, const void* x, int tin, void* y, int tout, const double* b, bool fp64,
                     hipStream_t s);
// TFPS (Sec. 2.2): y = A x (b null) or y = b - A x, computed in FP64; x, y
// FP32 (0) or FP64 (1); under a slot table x, y and b are workspace-relative.
void launch_tfps_apply(const Target& T, const void* x, int tin, void* y, int tout, const double* b,
                       hipStream_t s);
// psi at the cell centres, [N][cells] FP64, from the coefficients x
void launch_tfps_centres(const Target& T, const double* x, double* psi, hipStream_t s);
// host: the TFPS bases, tables and right-hand side of an operator whose
// scalar fields (grid, directions, S) are set
struct TfpsHost {
  std::vector<double> Lt, xi, chis, b;
  std::vector<double> sT, ux, uy;  // per cell sigma_T / eps; direction components
  std::vector<int> bid;
  int nbasis = 0;
};
TfpsHost tfps_build_host(const Operator& op, const std::vector<double>& dirs, const std::vector<double>& w,
                         const std::vector<double>& sT, const std::vector<double>& sA,
                         const std::vector<double>& qh, const double* inflow, size_t fstride);

// ATFPS (Sec. 2.3) on a TFPS operator: the three maps the device evaluates,
// each a sparse matrix and a constant (see atfps_setup.cpp).
struct HostCsr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> ptr, col;
  std::vector<double> val;
};
struct AtfpsHost {
  int64_t cells = 0, n_kept = 0, n_rows = 0, n_full = 0;
  int ndir = 0;
  HostCsr A, R, M;                 // compressed system, reconstruction, filtered-loss map
  std::vector<double> b, r0, c0;   // their constants
};
AtfpsHost atfps_build_host(const Operator& op, double delta);
struct DevCsr {
  int64_t nrows = 0, ncols = 0;
  const int64_t* ptr = nullptr;
  const int64_t* col = nullptr;
  const double* val = nullptr;
};
// y = c - A x (sub = true) or y = A x + c (sub = false); c may be null (zero)
void launch_csr(const DevCsr& A, const double* x, const double* c, bool sub, double* y, hipStream_t s);
// *out = ||v||_2 over n values: fixed-order two-stage sum, partials in part
// (device, kNorm2Parts doubles)
constexpr int kNorm2Parts = 1024;
void launch_norm2(const double* v, int64_t n, double* part, double* out, hipStream_t s);

// vscale (nullable, workspace-relative under a slot table): v is taken times
// vscale[0]; t16: t0 (or t) is stored as bfloat16 bits
void launch_lift(const Target& T, const Model& m, const double* v, const double* vscale, float* f0,
                 const float* ainv, float* t0, bool t16, hipStream_t s);
void launch_proj(const Target& T, const Model& m, const double* v, const double* vscale, const float* u0,
                 float* z, hipStream_t s);
void launch_scale_fields(const Slots& sl, const float* ainv, const float* f, float* t, int64_t count, bool t16,
                         hipStream_t s);
void launch_fill_f32(const Slots& sl, float* p, float v, int64_t count, hipStream_t s);
void launch_fill_f64(const Slots& sl, double* p, double v, int64_t count, hipStream_t s);
void launch_cast_f64_f32(const Slots& sl, const double* src, const double* scale, float* dst, int64_t count,
                         hipStream_t s);
void launch_copy_f64(const Slots& sl, const double* src, double* dst, int64_t count, hipStream_t s);

// CoeffNet (setup)
void launch_coef_conv(const float* in, int cin, const int in_dim[3], const float* w, const float* b,
                      float* out, int cout, const int out_dim[3], int dim, int stride, hipStream_t s);
void launch_head(const float* F, int c, const float* w, const float* b, float* out, int C,
                 int64_t P, hipStream_t s);

// Krylov (FP64).  Every array is per solve (workspace-relative under a slot
// table).
int krylov_blocks(int64_t n);
void launch_dots(const Slots& sl, const double* V, int64_t ldv, int nv, const double* w, int64_t n,
                 double* part, int nblk, hipStream_t s);
void launch_reduce(const Slots& sl, const double* part, int nblk, int nv, double* out, hipStream_t s);
// The Arnoldi step kernels below run under a slot table and take each
// slot's step j from its descriptor; jmax bounds j over the launch's slots
// (it picks the register budget).
// Lagged CGS2, first pass: V[j] <- (V[j] - sum_{i<j} h_i V_i) * fsc[0]
// (completing the current basis vector; for j = 0 the scaling of the
// residual), then part: V_i^T w for i <= j, with w = V[j + 1].
void launch_finish_dots(const Slots& sl, double* V, int64_t ldv, int jmax, const double* h, const double* fsc,
                        int64_t n, double* part, int nblk, hipStream_t s);
// Second pass, w = V[j + 1]: w <- w - V h; part: V^T w (first j + 1) and
// w.w (index j + 1)
void launch_updots(const Slots& sl, const double* V, int64_t ldv, int jmax, const double* h, int64_t n,
                   double* part, int nblk, hipStream_t s);
// Hessenberg column j, Givens, |g_{j+1}|/||b||; records the step in the
// slot's descriptor and ends the slot's cycle (live off, edge on) when the
// estimate meets rtol, the step limit is reached or breakdown occurs.
// A slot whose step exceeds jmax (the bound the launch was sized for) has
// its cycle discarded as a breakdown.
void launch_finish_step(const Slots& sl, const double* h1, const double* h2, int k, int jmax, double* H,
                        double* cs, double* sn, double* g, const double* bnorm, double* stat, hipStream_t s);
// beta = ||r|| from partial sums; g = beta e_1 (when given); stat[3] = stat[5]
// = 1/beta, stat[4] = beta.
void launch_start_cycle(const Slots& sl, const double* partn, int nblk, double* g, int k, double* stat,
                        hipStream_t s);
// jj: steps to combine; under a slot table each slot's own count is used
void launch_lsq(const Slots& sl, const double* H, const double* g, int jj, int k, double* y, hipStream_t s);
void launch_xupdate(const Slots& sl, double* x, const float* Z, int64_t ldz, const double* y, int jj,
                    int64_t n, hipStream_t s);
// At a cycle boundary (slots at the edge): the restart-or-finish decision
// from stat[4] = ||b - L x|| and bn[0] = ||b||, recorded in the descriptor.
void launch_decide(const Slots& sl, const double* stat, const double* bn, int k, hipStream_t s);

// kernel-class timing.  A sampled scope owns an event pair.  With ext =
// true the enclosed launch goes through launch_k, and the dispatch itself
// stamps the events around the kernel's execution (the interval a kernel
// trace reports); otherwise the events are recorded on the stream around
// everything the scope encloses.
struct ProfScope {
  int cls;
  hipStream_t s;
  double work = 0;   // algorithmic FLOPs (or bytes) of the enclosed launch
  double bytes = -1; // algorithmic bytes; < 0 means equal to work
  int key = 0;       // sub-class of the launch (conv: log2 of the output channels)
  bool ext;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ProfScope(int cls, hipStream_t s, bool ext = false);
  ~ProfScope();
};

// Thread-local state of the kernel-class timer: while a graph is being
// captured nothing is timed; inside a sampled (eager) Arnoldi step every
// launch of an enabled class is timed.
bool& prof_capturing();
bool& prof_force();
// Work multiplier of the launches timed while it is set: the number of
// slots they covered, filled in once the host knows it (negative until
// then; a null pointer means 1).
std::shared_ptr<double>& prof_scale();
bool& prof_quiet();    // batch bookkeeping launches outside sampled steps are not timed
int prof_stride();  // 0 when no class is being timed, else the smallest `every`

template <typename F, typename... Args>
inline void launch_k(F kernel, dim3 grid, dim3 block, uint32_t lds, hipStream_t s, const ProfScope& ps,
                     Args... args) {
  if (ps.e0 && ps.ext)
    hipExtLaunchKernelGGL(kernel, grid, block, lds, s, ps.e0, ps.e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
}

// solver internals shared with the server
struct SolveLayout {
  int k;
  int64_t n, ldv, ldz;
  int nblk;
  size_t off_x, off_b, off_V, off_Z, off_part1, off_part2, off_partn, off_small, off_mg, total;
  size_t mg_bytes;
};
// Per-solve workspace: iterate x and right-hand side b (FP64), the Krylov
// basis V (k + 1 FP64 vectors), the preconditioned vectors Z (k FP32
// vectors), partial sums, the small dense state and the V-cycle levels.
SolveLayout solve_layout(const Operator& op, const Model* m, int k, bool mgnet);
size_t precond_bytes(const Operator& op, const Model& m);
void validate_opts(const Operator& op, const Model* m, const rte_solve_opts* o);
void precond_apply(const Target& T, const Model& m, int kind, const double* v, float* z, char* ws,
                   hipStream_t s, const double* vscale = nullptr);

// Device tables of a batch: the slot descriptors and the per-slot report.
size_t batch_table_bytes(int capacity);

// A group of flexible GMRES(k) solves of one shape (Saad's right-
// preconditioned FGMRES with FP64 Arnoldi and an FP64 true residual at every
// restart) advanced together on one stream.  The group advances in ticks:
// a tick is the boundary launches (only when some slot waits at a cycle
// edge or a solve was admitted in it), one Arnoldi step of every live slot
// and a copy of the slot table to the host.  Each slot runs its own cycle
// at its own step, so a solve joins at the next tick and a restart costs
// its own slot one tick, not the group a synchronisation.  At most two
// ticks are in flight; the host reads each tick's table copy in order to
// admit, launch boundaries and copy finished results out.
class Batch {
 public:
  struct Finished {
    void* tag;
    rte_status status;
    rte_solve_stats stats;
  };
  Batch(const Operator& shape, const Model* m, int k, int precond, int capacity, char* tables, hipStream_t s);
  ~Batch();
  Batch(const Batch&) = delete;
  Batch& operator=(const Batch&) = delete;
  bool compatible(const Operator& op, const Model* m, int k, int precond) const;
  bool full() const;      // every slot is taken or promised to a waiting solve
  bool idle() const;      // nothing in flight, occupied, waiting or draining
  int members() const;    // occupied + waiting
  // A solve to join at the next tick; ws holds solve_layout bytes.
  void add(void* tag, const Operator& op, const rte_solve_opts& o, char* ws, double* out, double t_start);
  bool ready();           // the oldest tick in flight has completed (non-blocking)
  void wait();
  void advance();         // read the oldest completed tick, then keep two ticks in flight
  // Solves whose result has reached the caller's output buffer.
  void collect(std::vector<Finished>& out);
  // After a device error: waits for the stream and hands back every solve.
  void abandon(rte_status st, std::vector<Finished>& out);
  // The launches of one Arnoldi step of every live slot; jmax bounds the
  // slots' steps (one less than the register budget of the dot kernels).
  void step_body(int jmax, int zc, hipStream_t s);

 private:
  struct Event {  // one completion event shared by the solves emitted together
    hipEvent_t e = nullptr;
    ~Event() {
      if (e) (void)hipEventDestroy(e);
    }
  };
  struct Member {
    void* tag = nullptr;
    const Operator* op = nullptr;
    rte_solve_opts o{};
    char* ws = nullptr;
    double* out = nullptr;
    double t0 = 0, ms = 0;
    int slot = -1;
    int iters = 0, restarts = 0, steps_seen = 0;
    double rel = 0;
    int64_t since = 0;       // tick that admitted the solve
    int64_t bnd_tick = -1;   // last tick whose boundary launches cover the solve
    bool edge_pending = false;
    rte_status status = RTE_EAGAIN;
    std::shared_ptr<Event> copied;
  };
  void enqueue_tick();
  void boundary_launches(int zc);
  void admit(int z, SlotInit& in);
  void process(int64_t t);
  void fill();
  void finish_member(int z, const SlotDesc& d, SlotEmit& em);
  void upload_all();

  std::unique_ptr<Operator> shape_;  // geometry only: the first request's operator may be freed
  std::vector<int64_t> key_;
  const Model* m_;
  int k_, precond_, kind_, cap_;
  bool mg_, bj_;
  SolveLayout lay_;
  OpArrays rel_;
  SlotDesc* tab_;               // device [cap]
  SlotInit* dinit_;             // device [cap]: a tick's admissions
  SlotEmit* demit_;             // device [cap]: a tick's finished results
  hipStream_t s_;
  SlotDesc* hdesc_ = nullptr;   // pinned [cap]: all-off descriptors (reset)
  SlotInit* hinit_ = nullptr;   // pinned [2][cap], by tick parity
  SlotEmit* hemit_ = nullptr;   // pinned [2][cap], by the parity of the tick read
  SlotDesc* hsnap_ = nullptr;   // pinned [2][cap]: the table after each tick
  hipEvent_t ev_tick_[2] = {nullptr, nullptr};
  int tick_zc_[2] = {0, 0};
  std::shared_ptr<double> tick_scale_[2];
  std::vector<std::unique_ptr<Member>> slot_;  // occupant per slot
  std::vector<std::unique_ptr<Member>> waiting_, draining_;
  int64_t t_enq_ = 0, t_done_ = 0;  // ticks enqueued / read back
  int64_t snap_tick_ = -1;          // the last tick read back
  int snap_jmax_ = 0;               // largest step of a live slot in it
  int zc_ = 0;                      // slots the launches cover (grows while the batch is busy)
  bool graphs_ = true;
};

// Arnoldi-step graphs are keyed by everything their kernel arguments hold:
// the slot table, the model, the preconditioner, the restart length, the
// operator shape and the number of slots covered.  Freeing a model drops
// the graphs that reference its weights.
std::vector<hipGraphExec_t>* step_graphs(const void* tab, const Model* m, int precond, int k,
                                         const std::vector<int64_t>& shape, int zc);
void drop_step_graphs(const Model* m);
// A live batch marks its slot table in use: graphs of tables in use are
// never evicted.  Graphs of other tables stay cached (a later solve on the
// same workspace reuses them) up to a bounded number of keys, least
// recently used first out.
void step_graphs_hold(const void* tab);
void step_graphs_release(const void* tab);

}  // namespace rte

// Opaque handles of the C ABI.
struct rte_operator {
  std::unique_ptr<rte::Operator> op;
};
struct mgnet_model {
  std::unique_ptr<rte::Model> m;
};
struct rte_atfps {
  const rte::Operator* op = nullptr;
  rte::AtfpsHost host;
  rte::DevArena mem;
  rte::DevCsr A, R, M;
  double *b = nullptr, *r0 = nullptr, *c0 = nullptr;
  double* part = nullptr;  // partial sums of the loss norm (kNorm2Parts)
  int device = 0;
};


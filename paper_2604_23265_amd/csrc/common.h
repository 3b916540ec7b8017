// Internal declarations shared by the librte sources (not part of the ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
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
  std::vector<const float*> d_CW, d_CB, d_HAW, d_HAB, d_HIW, d_HIB;
  void ensure_on_device();  // uploads once, on the current device
  ~Model();
};

// --------------------------------------------------------- the operator ---
struct Operator {
  int dim = 2, nx = 0, ny = 0, nz = 1, ndir = 0, kernel = 0;
  int64_t cells = 0, n = 0;
  double h = 0, g = 0;
  int device = 0;
  std::vector<double> S;            // [N][N] host copy
  DevArena mem;
  double* b64 = nullptr;            // [n]
  float* sT32 = nullptr;            // sigma_T / eps            [cells]
  float* sA32 = nullptr;            // eps sigma_a              [cells]
  double* sT64 = nullptr;
  double* sA64 = nullptr;
  float* S32 = nullptr;             // [N][N]
  double* S64 = nullptr;
  float* dc32 = nullptr;            // per direction: |u_x|/h, |u_y|/h, |u_z|/h, sum  [N][4]
  double* dc64 = nullptr;
  int* dsgn = nullptr;              // per direction: sign(u_x), sign(u_y), sign(u_z)   [N][4]
  float* Sdiag32 = nullptr;         // S_mm                    [N]
  const Model* model = nullptr;     // CoeffNet fields were built for this model
  std::vector<float*> fa, fainv;    // per level [cells_l][C_l]
  int64_t level_cells(int l) const;
  int level_dim(int l, int axis) const;
};

// ------------------------------------------------------------ launchers ---
struct ApplyGeom {
  int N, nx, ny, nz;
  int64_t cells;
};

// y = L x (res = 0) or y = b - L x (res = 1).  tin/tout: 0 float, 1 double;
// compute precision follows `fp64`.
void launch_apply(const Operator& op, const void* x, int tin, void* y, int tout, const double* b,
                  bool fp64, hipStream_t s);

// MgNet pieces
// STORE_T: out = conv and out2 = a^{-1} (.) conv (a level's first smoothing input)
enum ConvMode { CONV_STORE = 0, CONV_ACCUM = 1, CONV_STORE_T = 2, CONV_RESID_R = 3, CONV_RESID_T = 4 };
enum MfmaKind { MFMA_F32 = 0, MFMA_BF16 = 1 };

struct ConvLaunch {
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
};
void launch_conv(const ConvLaunch& c, int kind, hipStream_t s);
void conv3_setup(ConvLaunch& c, int dim, const int in_dim[3], int stride);
void convT4_setup(ConvLaunch& c, int dim, const int in_dim[3]);

void launch_lift(const Operator& op, const Model& m, const double* v, float* f0, const float* ainv, float* t0,
                 hipStream_t s);
void launch_proj(const Operator& op, const Model& m, const double* v, const float* u0, float* z,
                 hipStream_t s);
void launch_scale_fields(const float* ainv, const float* f, float* t, int64_t count, hipStream_t s);
void launch_fill_f32(float* p, float v, int64_t count, hipStream_t s);
void launch_fill_f64(double* p, double v, int64_t count, hipStream_t s);
void launch_cast_f64_f32(const double* src, float* dst, int64_t count, hipStream_t s);
void launch_copy_f64(const double* src, double* dst, int64_t count, hipStream_t s);

// CoeffNet (setup)
void launch_coef_conv(const float* in, int cin, const int in_dim[3], const float* w, const float* b,
                      float* out, int cout, const int out_dim[3], int dim, int stride, hipStream_t s);
void launch_head(const float* F, int c, const float* w, const float* b, float* out, int C,
                 int64_t P, hipStream_t s);

// Krylov (FP64)
int krylov_blocks(int64_t n);
void launch_dots(const double* V, int64_t ldv, int nv, const double* w, int64_t n, double* part,
                 int nblk, hipStream_t s);
void launch_reduce(const double* part, int nblk, int nv, double* out, hipStream_t s);
// w <- w - V h; part: V^T w (first nv) and w.w (index nv)
void launch_updots(const double* V, int64_t ldv, int nv, const double* h, double* w, int64_t n,
                   double* part, int nblk, hipStream_t s);
// w <- (w - V h) * f[0]
void launch_update_scale(const double* V, int64_t ldv, int nv, const double* h, double* w, int64_t n,
                         const double* f, hipStream_t s);
void launch_finish_step(const double* h1, const double* h2, int j, int k, double* H, double* cs, double* sn,
                        double* g, const double* bnorm, double* stat, hipStream_t s);
void launch_scale_by(double* w, const double* stat_inv, int64_t n, hipStream_t s);
void launch_start_cycle(const double* partn, int nblk, double* g, int k, double* stat,
                        hipStream_t s);
void launch_lsq(const double* H, const double* g, int jj, int k, double* y, hipStream_t s);
void launch_xupdate(double* x, const float* Z, int64_t ldz, const double* y, int jj, int64_t n,
                    hipStream_t s);

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
  int64_t n;
  int nblk;
  size_t off_V, off_Z, off_part1, off_part2, off_partn, off_small, off_mg, total;
  size_t mg_bytes;
};
SolveLayout solve_layout(const Operator& op, const Model* m, int k, bool mgnet);
size_t precond_bytes(const Operator& op, const Model& m);
void validate_opts(const Operator& op, const Model* m, const rte_solve_opts* o);
void precond_apply(const Operator& op, const Model& m, int kind, const double* v, float* z,
                   char* ws, hipStream_t s);


// One flexible GMRES solve as a resumable state machine.  Work is enqueued
// on one stream; every host decision reads a small FP64 status block that
// the device copies into pinned host memory, and at most two Arnoldi steps
// are in flight ahead of the decision that may make the second one unused.
// rte_solve drives a run with blocking waits; the server interleaves many
// runs with non-blocking readiness checks.
class SolveRun {
 public:
  SolveRun(const Operator& op, const Model* m, const rte_solve_opts& o, char* ws, size_t ws_bytes,
           double* x, hipStream_t s);
  ~SolveRun();
  SolveRun(const SolveRun&) = delete;
  SolveRun& operator=(const SolveRun&) = delete;
  void start();
  bool ready();
  void wait();
  void advance();
  void step_body(int j, hipStream_t s);  // the kernels of Arnoldi step j
  bool done() const { return phase_ == DONE; }
  void fill_stats(rte_solve_stats* st) const;
  rte_status status() const { return status_; }

 private:
  enum Phase { BNORM, BETA, STEPS, FINAL, DONE };
  enum { SLOT_A = 0, SLOT_B = 1, SLOT_R = 2 };
  void enqueue_restart();
  void enqueue_step(int j);
  void read_into(int slot, const double* dev, int count);
  void finish(rte_status st);

  const Operator& op_;
  const Model* m_;
  rte_solve_opts o_;
  double* x_;
  hipStream_t s_;
  SolveLayout lay_;
  bool mg_;
  int kind_;
  const double* b_;
  double *V_, *part1_, *part2_, *partn_;
  float* Z_;
  char* mgws_;
  double *H_, *g_, *cs_, *sn_, *y_, *h1_, *h2_, *stat_, *bn_;
  double* host_ = nullptr;   // pinned [3][8]
  hipEvent_t ev_[3] = {nullptr, nullptr, nullptr};
  Phase phase_ = BNORM;
  int wait_slot_ = SLOT_R;
  int j_wait_ = 0, j_enq_ = 0;
  int iters_ = 0, restarts_ = 0, stall_ = 0;
  double bnorm_ = 0, prev_ = 0, rel_ = 0;
  rte_status status_ = RTE_ENOCONV;
  double t0_ = 0, ms_ = 0;
  bool graphs_ = true;
  std::vector<hipGraphExec_t>* gcache_ = nullptr;  // per-step graphs for this workspace
};

// Graphs of Arnoldi steps, keyed by everything their kernel arguments hold;
// dropped when the operator they reference is freed.
std::vector<hipGraphExec_t>* step_graphs(const Operator* op, const Model* m, int precond, const char* ws,
                                         const double* x, const double* b, int k);
void drop_step_graphs(const Operator* op);

}  // namespace rte

// Opaque handles of the C ABI.
struct rte_operator {
  std::unique_ptr<rte::Operator> op;
};
struct mgnet_model {
  std::unique_ptr<rte::Model> m;
};


// MgNet V-cycle orchestration and the flexible GMRES driver.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <tuple>

#include "common.h"

namespace rte {

namespace {
size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

// Level activations of one V-cycle: f_l (right-hand side), u_l (iterate),
// t_l (scratch: modulated residual / residual), each [cells_l][C_l] FP32.
size_t precond_bytes(const Operator& op, const Model& m) {
  size_t total = 0;
  for (int l = 0; l < m.levels; ++l) total += 3 * align256(size_t(op.level_cells(l)) * (m.c0 << l) * 4);
  return total;
}

// z = M(v), the V-cycle of Sec. 3.3 in the reading documented with the
// oracle: lift, nu_pre smoothing steps and a stride-2 restriction of the
// residual per level, nu_coarse steps on the coarsest level, then per level
// a stride-2 transposed-conv prolongation added to u and nu_post steps,
// and the projection plus the diagonal skip.  A smoothing step is two
// launches: t = a^{-1} (.) (f - A * u - a (.) u) and u += B * t.
void precond_apply(const Operator& op, const Model& m, int kind, const double* v, float* z, char* ws,
                   hipStream_t s) {
  ProfScope ps(RTE_K_PRECOND, s);
  const int L = m.levels;
  std::vector<float*> f(L), u(L), t(L);
  std::vector<int64_t> P(L);
  std::vector<int> C(L);
  char* p = ws;
  for (int l = 0; l < L; ++l) {
    P[l] = op.level_cells(l);
    C[l] = m.c0 << l;
    const size_t b = align256(size_t(P[l]) * C[l] * 4);
    f[l] = reinterpret_cast<float*>(p); p += b;
    u[l] = reinterpret_cast<float*>(p); p += b;
    t[l] = reinterpret_cast<float*>(p); p += b;
  }
  auto dims = [&](int l, int d[3]) {
    for (int a = 0; a < 3; ++a) d[a] = op.level_dim(l, a);
  };
  auto conv_same = [&](int l, const float* in, const ConvW& w, float* out, int mode) {
    ConvLaunch c{};
    int d[3];
    dims(l, d);
    conv3_setup(c, op.dim, d, 1);
    c.in = in; c.cin = w.cin; c.w = &w; c.out = out; c.cout = w.cout; c.mode = mode;
    c.f = f[l]; c.a = op.fa[l]; c.ainv = op.fainv[l];
    launch_conv(c, kind, s);
  };
  // uz[l]: u_l is still zero; tready[l]: t_l already holds a^{-1} (.) f_l,
  // written by the producer of f_l (lift or restriction epilogue)
  std::vector<bool> uz(L, true), tready(L, false);
  auto first_steps = [&](int l) {
    return l < L - 1 ? int(m.Bpre[l].size()) : int(m.Bc.size());
  };
  auto smooth = [&](int l, const ConvW& B) {
    if (uz[l]) {
      if (!tready[l]) launch_scale_fields(op.fainv[l], f[l], t[l], P[l] * C[l], s);
      tready[l] = false;
      conv_same(l, t[l], B, u[l], CONV_STORE);
      uz[l] = false;
    } else {
      conv_same(l, u[l], m.A[l], t[l], CONV_RESID_T);
      conv_same(l, t[l], B, u[l], CONV_ACCUM);
    }
  };

  const bool want0 = first_steps(0) > 0;
  launch_lift(op, m, v, f[0], want0 ? op.fainv[0] : nullptr, want0 ? t[0] : nullptr, s);
  tready[0] = want0;
  for (int l = 0; l < L - 1; ++l) {
    uz[l] = true;
    for (const ConvW& B : m.Bpre[l]) smooth(l, B);
    const float* rin = f[l];
    if (!uz[l]) {
      conv_same(l, u[l], m.A[l], t[l], CONV_RESID_R);
      rin = t[l];
    }
    ConvLaunch c{};
    int d[3];
    dims(l, d);
    conv3_setup(c, op.dim, d, 2);
    const bool want = first_steps(l + 1) > 0;
    c.in = rin; c.cin = m.R[l].cin; c.w = &m.R[l]; c.out = f[l + 1]; c.cout = m.R[l].cout;
    c.mode = want ? CONV_STORE_T : CONV_STORE;
    c.out2 = want ? t[l + 1] : nullptr;
    c.ainv = op.fainv[l + 1];
    launch_conv(c, kind, s);
    tready[l + 1] = want;
  }
  uz[L - 1] = true;
  for (const ConvW& B : m.Bc) smooth(L - 1, B);
  if (uz[L - 1]) launch_fill_f32(u[L - 1], 0.f, P[L - 1] * C[L - 1], s);
  for (int l = L - 2; l >= 0; --l) {
    ConvLaunch c{};
    int d[3];
    dims(l + 1, d);
    convT4_setup(c, op.dim, d);
    c.in = u[l + 1]; c.cin = m.Pr[l].cin; c.w = &m.Pr[l]; c.out = u[l]; c.cout = m.Pr[l].cout;
    c.mode = uz[l] ? CONV_STORE : CONV_ACCUM;
    launch_conv(c, kind, s);
    uz[l] = false;
    for (const ConvW& B : m.Bpost[l]) smooth(l, B);
  }
  if (uz[0]) launch_fill_f32(u[0], 0.f, P[0] * C[0], s);
  launch_proj(op, m, v, u[0], z, s);
}

constexpr int HMAX = 65;

SolveLayout solve_layout(const Operator& op, const Model* m, int k, bool mgnet) {
  SolveLayout L{};
  L.k = k;
  L.n = op.n;
  L.nblk = krylov_blocks(op.n);
  size_t off = 0;
  L.off_V = off; off += align256(size_t(k + 1) * op.n * 8);
  L.off_Z = off; off += align256(size_t(k) * op.n * 4);
  L.off_part1 = off; off += align256(size_t(L.nblk) * HMAX * 8);
  L.off_part2 = off; off += align256(size_t(L.nblk) * HMAX * 8);
  L.off_partn = off; off += align256(size_t(L.nblk) * HMAX * 8);
  L.off_small = off; off += align256(size_t(k + 1) * k * 8 + size_t(6 * HMAX + 32) * 8);
  L.mg_bytes = (mgnet && m) ? precond_bytes(op, *m) : 0;
  L.off_mg = off; off += L.mg_bytes;
  L.total = off;
  return L;
}

namespace {

struct GraphKey {
  const Operator* op;
  const Model* m;
  int precond;
  const char* ws;
  const double* x;
  const double* b;
  int k;
  bool operator<(const GraphKey& o) const {
    return std::tie(op, m, precond, ws, x, b, k) < std::tie(o.op, o.m, o.precond, o.ws, o.x, o.b, o.k);
  }
};

std::mutex g_graph_mu;
std::map<GraphKey, std::unique_ptr<std::vector<hipGraphExec_t>>>& graph_map() {
  static auto* m = new std::map<GraphKey, std::unique_ptr<std::vector<hipGraphExec_t>>>();
  return *m;
}

std::atomic<int64_t> g_steps{0};  // Arnoldi steps enqueued by every solve (timer sampling)

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

std::vector<hipGraphExec_t>* step_graphs(const Operator* op, const Model* m, int precond, const char* ws,
                                         const double* x, const double* b, int k) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto& slot = graph_map()[GraphKey{op, m, precond, ws, x, b, k}];
  if (!slot) slot.reset(new std::vector<hipGraphExec_t>(size_t(k), nullptr));
  return slot.get();
}

void drop_step_graphs(const Operator* op) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto& mp = graph_map();
  for (auto it = mp.begin(); it != mp.end();) {
    if (it->first.op == op) {
      for (hipGraphExec_t e : *it->second)
        if (e) (void)hipGraphExecDestroy(e);
      it = mp.erase(it);
    } else {
      ++it;
    }
  }
}

void validate_opts(const Operator& op, const Model* m, const rte_solve_opts* o) {
  RTE_REQUIRE(o != nullptr, RTE_EINVAL, "null solve options");
  RTE_REQUIRE(o->restart >= 1 && o->restart <= 64, RTE_EINVAL, "restart must be in [1, 64]");
  RTE_REQUIRE(std::isfinite(o->rtol) && o->rtol > 0, RTE_EINVAL, "rtol must be positive");
  RTE_REQUIRE(o->max_iters >= 1, RTE_EINVAL, "max_iters must be >= 1");
  RTE_REQUIRE(o->precond >= RTE_PC_NONE && o->precond <= RTE_PC_MGNET_FP32, RTE_EINVAL,
              "unknown preconditioner");
  if (o->precond != RTE_PC_NONE) {
    RTE_REQUIRE(m != nullptr, RTE_EINVAL, "MgNet preconditioning needs a model");
    RTE_REQUIRE(op.model == m, RTE_EINVAL, "operator was not built with this model (CoeffNet fields missing)");
  }
}

// Flexible GMRES(k), right preconditioned (Saad): inner steps in reduced
// precision (FP32 operator apply, FP32 or BF16 MgNet), orthogonalisation and
// least squares in FP64, and the true residual b - L x recomputed in FP64
// at every restart (iterative refinement on the FP64 iterate x).
SolveRun::SolveRun(const Operator& op, const Model* m, const rte_solve_opts& o, char* ws, size_t ws_bytes,
                   double* x, hipStream_t s)
    : op_(op), m_(m), o_(o), x_(x), s_(s) {
  validate_opts(op, m, &o);
  mg_ = o.precond != RTE_PC_NONE;
  kind_ = o.precond == RTE_PC_MGNET_FP32 ? MFMA_F32 : MFMA_BF16;
  lay_ = solve_layout(op, m, o.restart, mg_);
  RTE_REQUIRE(ws != nullptr && x != nullptr, RTE_EINVAL, "null workspace or output");
  RTE_REQUIRE(ws_bytes >= lay_.total, RTE_ENOMEM, "workspace too small: need " + std::to_string(lay_.total) + " bytes");
  RTE_REQUIRE((reinterpret_cast<uintptr_t>(ws) & 255) == 0, RTE_EINVAL, "workspace must be 256-byte aligned");
  if (mg_) const_cast<Model*>(m)->ensure_on_device();
  const int k = o.restart;
  V_ = reinterpret_cast<double*>(ws + lay_.off_V);
  Z_ = reinterpret_cast<float*>(ws + lay_.off_Z);
  part1_ = reinterpret_cast<double*>(ws + lay_.off_part1);
  part2_ = reinterpret_cast<double*>(ws + lay_.off_part2);
  partn_ = reinterpret_cast<double*>(ws + lay_.off_partn);
  double* p = reinterpret_cast<double*>(ws + lay_.off_small);
  H_ = p; p += size_t(k + 1) * k;
  g_ = p; p += HMAX;
  cs_ = p; p += HMAX;
  sn_ = p; p += HMAX;
  y_ = p; p += HMAX;
  h1_ = p; p += HMAX;
  h2_ = p; p += HMAX;
  stat_ = p; p += 16;
  bn_ = p;
  mgws_ = ws + lay_.off_mg;
  b_ = o.b ? o.b : op.b64;
  const char* env = std::getenv("RTE_GRAPHS");
  graphs_ = !(env && env[0] == '0');
  if (graphs_) gcache_ = step_graphs(&op, m, o.precond, ws, x, b_, k);
  RTE_HIP(hipHostMalloc(reinterpret_cast<void**>(&host_), 3 * 8 * sizeof(double), hipHostMallocDefault));
  for (auto& e : ev_) RTE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

SolveRun::~SolveRun() {
  for (auto& e : ev_)
    if (e) (void)hipEventDestroy(e);
  if (host_) (void)hipHostFree(host_);
}

void SolveRun::read_into(int slot, const double* dev, int count) {
  RTE_HIP(hipMemcpyAsync(host_ + 8 * slot, dev, size_t(count) * 8, hipMemcpyDeviceToHost, s_));
  RTE_HIP(hipEventRecord(ev_[slot], s_));
}

void SolveRun::start() {
  t0_ = now_ms();
  const int64_t n = op_.n;
  if (o_.x0)
    launch_copy_f64(o_.x0, x_, n, s_);
  else
    launch_fill_f64(x_, 0.0, n, s_);
  launch_dots(b_, n, 1, b_, n, partn_, lay_.nblk, s_);
  launch_start_cycle(partn_, lay_.nblk, nullptr, lay_.k, stat_, s_);
  launch_copy_f64(stat_ + 4, bn_, 1, s_);
  read_into(SLOT_R, stat_ + 4, 1);
  phase_ = BNORM;
  wait_slot_ = SLOT_R;
}

bool SolveRun::ready() {
  if (phase_ == DONE) return true;
  hipError_t e = hipEventQuery(ev_[wait_slot_]);
  if (e == hipErrorNotReady) return false;
  RTE_HIP(e);
  return true;
}

void SolveRun::wait() {
  if (phase_ == DONE) return;
  RTE_HIP(hipEventSynchronize(ev_[wait_slot_]));
}

void SolveRun::enqueue_restart() {
  const int64_t n = op_.n;
  launch_apply(op_, x_, 1, V_, 1, b_, true, s_);  // r = b - L x in FP64
  launch_dots(V_, n, 1, V_, n, partn_, lay_.nblk, s_);
  launch_start_cycle(partn_, lay_.nblk, g_, lay_.k, stat_, s_);
  read_into(SLOT_R, stat_, 5);
  wait_slot_ = SLOT_R;
}

// Arnoldi step j: z_j = M(v_j); w = L z_j; CGS2 against v_0..v_j; Givens.
void SolveRun::step_body(int j, hipStream_t s) {
  const int64_t n = op_.n;
  const int nb = lay_.nblk, k = lay_.k;
  const double* Vj = V_ + size_t(j) * n;
  double* Vn = V_ + size_t(j + 1) * n;
  float* Zj = Z_ + size_t(j) * n;
  if (mg_)
    precond_apply(op_, *m_, kind_, Vj, Zj, mgws_, s);
  else
    launch_cast_f64_f32(Vj, Zj, n, s);
  launch_apply(op_, Zj, 0, Vn, 1, nullptr, false, s);
  // CGS2 in three passes over V: h1 = V^T w; w1 = w - V h1 with h2 = V^T w1
  // and ||w1||^2; then v_{j+1} = (w1 - V h2) / ||w1 - V h2||
  launch_dots(V_, n, j + 1, Vn, n, part1_, nb, s);
  launch_reduce(part1_, nb, j + 1, h1_, s);
  launch_updots(V_, n, j + 1, h1_, Vn, n, part2_, nb, s);
  launch_reduce(part2_, nb, j + 2, h2_, s);
  launch_finish_step(h1_, h2_, j, k, H_, cs_, sn_, g_, bn_, stat_, s);
  launch_update_scale(V_, n, j + 1, h2_, Vn, n, stat_ + 3, s);
}

namespace {

// Capture the kernels of one Arnoldi step on a private stream (nothing runs
// during capture) and instantiate them as a graph.
hipGraphExec_t capture_step(SolveRun& run, int j) {
  thread_local hipStream_t cap = nullptr;
  if (!cap) RTE_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  prof_capturing() = true;
  hipGraph_t g = nullptr;
  RTE_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  try {
    run.step_body(j, cap);
  } catch (...) {
    (void)hipStreamEndCapture(cap, &g);
    if (g) (void)hipGraphDestroy(g);
    prof_capturing() = false;
    throw;
  }
  prof_capturing() = false;
  RTE_HIP(hipStreamEndCapture(cap, &g));
  hipGraphExec_t e = nullptr;
  hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  RTE_HIP(err);
  return e;
}

}  // namespace

// Replays the step's graph (captured on first use for this workspace);
// while the kernel-class timer is on, one step in `every` runs eagerly with
// all of its launches of the enabled classes timed.
void SolveRun::enqueue_step(int j) {
  const int stride = prof_stride();
  const bool sample = stride > 0 && (g_steps.fetch_add(1) % stride) == 0;
  if (!graphs_ || sample) {
    prof_force() = sample;
    try {
      step_body(j, s_);
    } catch (...) {
      prof_force() = false;
      throw;
    }
    prof_force() = false;
  } else {
    hipGraphExec_t& ge = (*gcache_)[j];
    if (!ge) ge = capture_step(*this, j);
    RTE_HIP(hipGraphLaunch(ge, s_));
  }
  read_into(j % 2, stat_, 2);
  j_enq_ = j + 1;
}

void SolveRun::finish(rte_status st) {
  status_ = st;
  phase_ = DONE;
  RTE_HIP(hipStreamSynchronize(s_));
  ms_ = now_ms() - t0_;
}

void SolveRun::advance() {
  if (phase_ == DONE) return;
  const double* h = host_ + 8 * wait_slot_;
  switch (phase_) {
    case BNORM: {
      bnorm_ = h[0];
      if (!std::isfinite(bnorm_)) fail(RTE_EINVAL, "right-hand side is not finite");
      if (bnorm_ == 0.0) {
        launch_fill_f64(x_, 0.0, op_.n, s_);
        rel_ = 0;
        finish(RTE_OK);
        return;
      }
      prev_ = INFINITY;
      enqueue_restart();
      phase_ = BETA;
      return;
    }
    case BETA: {
      const double beta = h[4];
      rel_ = beta / bnorm_;
      if (!std::isfinite(beta)) return finish(RTE_EBREAKDOWN);
      if (rel_ <= o_.rtol) return finish(RTE_OK);
      if (iters_ >= o_.max_iters) return finish(RTE_ENOCONV);
      if (beta >= prev_ * (1.0 - 1e-3)) {
        if (++stall_ >= 3) return finish(RTE_ENOCONV);
      } else {
        stall_ = 0;
      }
      prev_ = beta;
      launch_scale_by(V_, stat_ + 3, op_.n, s_);
      enqueue_step(0);
      if (lay_.k > 1) enqueue_step(1);
      j_wait_ = 0;
      wait_slot_ = 0;
      phase_ = STEPS;
      return;
    }
    case STEPS: {
      const double est = h[0];
      const int flags = int(h[1]);
      ++iters_;
      const int j = j_wait_;
      if (flags & 1) {
        // non-finite: keep the iterate of the last completed cycle
        --iters_;
        enqueue_restart();
        phase_ = FINAL;
        return;
      }
      const bool stop = (flags & 2) || est <= o_.rtol || iters_ >= o_.max_iters || j + 1 == lay_.k;
      if (stop) {
        // a speculative step j + 1 may still be queued: it writes only column
        // j + 1 of H, g[j + 1 ..], V_{j + 2} and Z_{j + 1}, none of which the
        // update below reads
        launch_lsq(H_, g_, j + 1, lay_.k, y_, s_);
        launch_xupdate(x_, Z_, op_.n, y_, j + 1, op_.n, s_);
        ++restarts_;
        enqueue_restart();
        phase_ = BETA;
        return;
      }
      j_wait_ = j + 1;
      wait_slot_ = j_wait_ % 2;
      if (j + 2 < lay_.k && j_enq_ == j + 2) enqueue_step(j + 2);
      return;
    }
    case FINAL: {
      rel_ = h[4] / bnorm_;
      return finish(RTE_EBREAKDOWN);
    }
    default:
      return;
  }
}

void SolveRun::fill_stats(rte_solve_stats* st) const {
  if (!st) return;
  st->iterations = iters_;
  st->restarts = restarts_;
  st->converged = status_ == RTE_OK;
  st->status = status_;
  st->rel_residual = rel_;
  st->ms_total = ms_;
}

}  // namespace rte

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
void precond_apply(const Target& T, const Model& m, int kind, const double* v, float* z, char* ws,
                   hipStream_t s, const double* vscale) {
  ProfScope ps(RTE_K_PRECOND, s);
  const Operator& op = *T.op;
  const Slots& sl = T.sl;
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
    c.sl = sl;
    c.in = in; c.cin = w.cin; c.w = &w; c.out = out; c.cout = w.cout; c.mode = mode;
    c.f = f[l]; c.a = T.arr.fa[l]; c.ainv = T.arr.fainv[l];
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
      if (!tready[l]) launch_scale_fields(sl, T.arr.fainv[l], f[l], t[l], P[l] * C[l], s);
      tready[l] = false;
      conv_same(l, t[l], B, u[l], CONV_STORE);
      uz[l] = false;
    } else {
      conv_same(l, u[l], m.A[l], t[l], CONV_RESID_T);
      conv_same(l, t[l], B, u[l], CONV_ACCUM);
    }
  };

  const bool want0 = first_steps(0) > 0;
  launch_lift(T, m, v, vscale, f[0], want0 ? T.arr.fainv[0] : nullptr, want0 ? t[0] : nullptr, s);
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
    c.sl = sl;
    const bool want = first_steps(l + 1) > 0;
    c.in = rin; c.cin = m.R[l].cin; c.w = &m.R[l]; c.out = f[l + 1]; c.cout = m.R[l].cout;
    c.mode = want ? CONV_STORE_T : CONV_STORE;
    c.out2 = want ? t[l + 1] : nullptr;
    c.ainv = T.arr.fainv[l + 1];
    launch_conv(c, kind, s);
    tready[l + 1] = want;
  }
  uz[L - 1] = true;
  for (const ConvW& B : m.Bc) smooth(L - 1, B);
  if (uz[L - 1]) launch_fill_f32(sl, u[L - 1], 0.f, P[L - 1] * C[L - 1], s);
  for (int l = L - 2; l >= 0; --l) {
    ConvLaunch c{};
    int d[3];
    dims(l + 1, d);
    convT4_setup(c, op.dim, d);
    c.sl = sl;
    c.in = u[l + 1]; c.cin = m.Pr[l].cin; c.w = &m.Pr[l]; c.out = u[l]; c.cout = m.Pr[l].cout;
    c.mode = uz[l] ? CONV_STORE : CONV_ACCUM;
    launch_conv(c, kind, s);
    uz[l] = false;
    for (const ConvW& B : m.Bpost[l]) smooth(l, B);
  }
  if (uz[0]) launch_fill_f32(sl, u[0], 0.f, P[0] * C[0], s);
  launch_proj(T, m, v, vscale, u[0], z, s);
}

constexpr int HMAX = 65;

namespace {
template <class T>
T* off(size_t o) {
  return reinterpret_cast<T*>(uintptr_t(o));
}
}  // namespace

SolveLayout solve_layout(const Operator& op, const Model* m, int k, bool mgnet) {
  SolveLayout L{};
  L.k = k;
  L.n = op.n;
  L.nblk = krylov_blocks(op.n);
  // nothing sits at offset 0: under a slot table a zero offset would read
  // as a null argument
  size_t off = 256;
  L.off_x = off; off += align256(size_t(op.n) * 8);
  L.off_b = off; off += align256(size_t(op.n) * 8);
  // basis vectors sit ldv (ldz) elements apart: a multiple of 256 bytes
  // plus 256, so the same element of successive vectors does not fall on
  // the same HBM channel (a power-of-two spacing would)
  L.ldv = ((op.n + 31) / 32) * 32 + 32;
  L.ldz = ((op.n + 63) / 64) * 64 + 64;
  L.off_V = off; off += align256(size_t(k + 1) * L.ldv * 8);
  L.off_Z = off; off += align256(size_t(k) * L.ldz * 4);
  L.off_part1 = off; off += align256(size_t(L.nblk) * HMAX * 8);
  L.off_part2 = off; off += align256(size_t(L.nblk) * HMAX * 8);
  L.off_partn = off; off += align256(size_t(L.nblk) * HMAX * 8);
  L.off_small = off; off += align256(size_t(k + 1) * k * 8 + size_t(6 * HMAX + 32) * 8);
  L.mg_bytes = (mgnet && m) ? precond_bytes(op, *m) : 0;
  L.off_mg = off; off += L.mg_bytes;
  L.total = off;
  return L;
}

size_t batch_table_bytes(int capacity) {
  return align256(size_t(capacity) * sizeof(SlotDesc)) + align256(size_t(capacity) * 8 * sizeof(double));
}

namespace {

// Offsets of the small dense state inside off_small.
struct Small {
  size_t H, g, cs, sn, y, h1, h2, stat, bn;
};
Small small_of(const SolveLayout& L) {
  Small q;
  size_t p = L.off_small;
  q.H = p; p += size_t(L.k + 1) * L.k * 8;
  q.g = p; p += HMAX * 8;
  q.cs = p; p += HMAX * 8;
  q.sn = p; p += HMAX * 8;
  q.y = p; p += HMAX * 8;
  q.h1 = p; p += HMAX * 8;
  q.h2 = p; p += HMAX * 8;
  q.stat = p; p += 16 * 8;
  q.bn = p;
  return q;
}

struct GraphKey {
  const void* tab;
  const Model* m;
  int precond, k, zc;
  std::vector<int64_t> shape;
  bool operator<(const GraphKey& o) const {
    return std::tie(tab, m, precond, k, zc, shape) < std::tie(o.tab, o.m, o.precond, o.k, o.zc, o.shape);
  }
};

std::mutex g_graph_mu;
std::map<GraphKey, std::unique_ptr<std::vector<hipGraphExec_t>>>& graph_map() {
  static auto* m = new std::map<GraphKey, std::unique_ptr<std::vector<hipGraphExec_t>>>();
  return *m;
}

std::atomic<int64_t> g_steps{0};  // Arnoldi steps enqueued by every batch (timer sampling)

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

std::vector<hipGraphExec_t>* step_graphs(const void* tab, const Model* m, int precond, int k,
                                         const std::vector<int64_t>& shape, int zc) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto& slot = graph_map()[GraphKey{tab, m, precond, k, zc, shape}];
  if (!slot) slot.reset(new std::vector<hipGraphExec_t>(size_t(k), nullptr));
  return slot.get();
}

void drop_step_graphs(const Model* m) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto& mp = graph_map();
  for (auto it = mp.begin(); it != mp.end();) {
    if (it->first.m == m) {
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
  RTE_REQUIRE(o->precond >= RTE_PC_NONE && o->precond <= RTE_PC_BLOCK_JACOBI, RTE_EINVAL,
              "unknown preconditioner");
  if (o->precond == RTE_PC_BLOCK_JACOBI)
    RTE_REQUIRE(op.ndir <= 64, RTE_EINVAL, "Block-Jacobi supports up to 64 directions");
  if (o->precond == RTE_PC_MGNET_BF16 || o->precond == RTE_PC_MGNET_FP32) {
    RTE_REQUIRE(m != nullptr, RTE_EINVAL, "MgNet preconditioning needs a model");
    RTE_REQUIRE(op.model == m, RTE_EINVAL, "operator was not built with this model (CoeffNet fields missing)");
  }
}

Batch::Batch(const Operator& shape, const Model* m, int k, int precond, int capacity, char* tables,
             hipStream_t s)
    : shape_(shape), key_(shape.shape_key()), m_(m), k_(k), precond_(precond), cap_(capacity), s_(s) {
  RTE_REQUIRE(capacity >= 1 && capacity <= 64, RTE_EINVAL, "batch capacity must be in [1, 64]");
  RTE_REQUIRE(tables != nullptr && (reinterpret_cast<uintptr_t>(tables) & 255) == 0, RTE_EINVAL,
              "batch tables must be 256-byte aligned");
  mg_ = precond == RTE_PC_MGNET_BF16 || precond == RTE_PC_MGNET_FP32;
  bj_ = precond == RTE_PC_BLOCK_JACOBI;
  kind_ = precond == RTE_PC_MGNET_FP32 ? MFMA_F32 : MFMA_BF16;
  lay_ = solve_layout(shape, m, k, mg_);
  rel_ = shape.relative();
  tab_ = reinterpret_cast<SlotDesc*>(tables);
  rep_ = reinterpret_cast<double*>(tables + align256(size_t(capacity) * sizeof(SlotDesc)));
  if (mg_) const_cast<Model*>(m)->ensure_on_device();
  const char* env = std::getenv("RTE_GRAPHS");
  graphs_ = !(env && env[0] == '0');
  slot_.resize(size_t(capacity));
  RTE_HIP(hipHostMalloc(reinterpret_cast<void**>(&hdesc_), size_t(capacity) * sizeof(SlotDesc),
                        hipHostMallocDefault));
  RTE_HIP(hipHostMalloc(reinterpret_cast<void**>(&hsnap_), 2 * size_t(capacity) * sizeof(SlotDesc),
                        hipHostMallocDefault));
  RTE_HIP(hipHostMalloc(reinterpret_cast<void**>(&hrep_), size_t(capacity) * 8 * sizeof(double),
                        hipHostMallocDefault));
  std::memset(hdesc_, 0, size_t(capacity) * sizeof(SlotDesc));
  std::memset(hsnap_, 0, 2 * size_t(capacity) * sizeof(SlotDesc));
  std::memset(hrep_, 0, size_t(capacity) * 8 * sizeof(double));
  for (auto& e : ev_step_) RTE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  RTE_HIP(hipEventCreateWithFlags(&ev_rep_, hipEventDisableTiming));
  upload_all();
}

Batch::~Batch() {
  (void)hipStreamSynchronize(s_);
  for (auto* v : {&waiting_, &draining_})
    for (auto& mb : *v)
      if (mb && mb->copied) (void)hipEventDestroy(mb->copied);
  for (auto& mb : slot_)
    if (mb && mb->copied) (void)hipEventDestroy(mb->copied);
  for (auto& e : ev_step_)
    if (e) (void)hipEventDestroy(e);
  if (ev_rep_) (void)hipEventDestroy(ev_rep_);
  if (hdesc_) (void)hipHostFree(hdesc_);
  if (hsnap_) (void)hipHostFree(hsnap_);
  if (hrep_) (void)hipHostFree(hrep_);
}

bool Batch::compatible(const Operator& op, const Model* m, int k, int precond) const {
  return m == m_ && k == k_ && precond == precond_ && op.shape_key() == key_;
}

int Batch::members() const {
  int c = int(waiting_.size());
  for (auto& mb : slot_)
    if (mb) ++c;
  return c;
}

bool Batch::full() const { return members() >= cap_; }

bool Batch::idle() const { return phase_ == IDLE && members() == 0 && draining_.empty(); }

void Batch::upload(int z) {
  RTE_HIP(hipMemcpyAsync(tab_ + z, hdesc_ + z, sizeof(SlotDesc), hipMemcpyHostToDevice, s_));
}

void Batch::upload_all() {
  RTE_HIP(hipMemcpyAsync(tab_, hdesc_, size_t(cap_) * sizeof(SlotDesc), hipMemcpyHostToDevice, s_));
}

void Batch::add(void* tag, const Operator& op, const rte_solve_opts& o, char* ws, double* out, double t_start) {
  RTE_REQUIRE(o.restart == k_ && o.precond == precond_ && op.shape_key() == key_ && (!mg_ || op.model == m_),
              RTE_EINVAL, "solve does not match the batch");
  RTE_REQUIRE(!full(), RTE_EINVAL, "batch is full");
  RTE_REQUIRE(ws && out && (reinterpret_cast<uintptr_t>(ws) & 255) == 0, RTE_EINVAL,
              "bad workspace or output");
  std::unique_ptr<Member> mb(new Member());
  mb->tag = tag;
  mb->op = &op;
  mb->o = o;
  mb->ws = ws;
  mb->out = out;
  mb->t0 = t_start;
  waiting_.push_back(std::move(mb));
  if (phase_ == IDLE) boundary();
}

// Cycle boundary: admit waiting solves into free slots, then for every
// occupied slot combine the finished cycle's steps into x (x += Z y), form
// the FP64 true residual r = b - L x as v_0, and report beta = ||r|| and
// ||b|| to the host.
namespace {
struct Quiet {
  Quiet() { prof_quiet() = true; }
  ~Quiet() { prof_quiet() = false; }
};
}  // namespace

void Batch::boundary() {
  Quiet quiet;
  const int64_t n = lay_.n;
  for (int z = 0; z < cap_ && !waiting_.empty(); ++z) {
    if (slot_[z]) continue;
    std::unique_ptr<Member> mb = std::move(waiting_.front());
    waiting_.erase(waiting_.begin());
    double* x = reinterpret_cast<double*>(mb->ws + lay_.off_x);
    double* b = reinterpret_cast<double*>(mb->ws + lay_.off_b);
    if (mb->o.x0)
      RTE_HIP(hipMemcpyAsync(x, mb->o.x0, size_t(n) * 8, hipMemcpyDeviceToDevice, s_));
    else
      launch_fill_f64(Slots{}, x, 0.0, n, s_);
    const double* bsrc = mb->o.b ? static_cast<const double*>(mb->o.b) : mb->op->a.b64;
    RTE_HIP(hipMemcpyAsync(b, bsrc, size_t(n) * 8, hipMemcpyDeviceToDevice, s_));
    SlotDesc d{};
    d.ws = reinterpret_cast<uint64_t>(mb->ws);
    d.op = reinterpret_cast<uint64_t>(mb->op->block);
    d.occupied = 1;
    d.rtol = mb->o.rtol;
    hdesc_[z] = d;
    upload(z);
    mb->slot = z;
    slot_[z] = std::move(mb);
  }
  zc_ = 0;
  for (int z = 0; z < cap_; ++z)
    if (slot_[z]) zc_ = z + 1;
  if (zc_ == 0) {
    phase_ = IDLE;
    return;
  }
  const Slots so = slots(1);
  const Target T{&shape_, rel_, so};
  const Small q = small_of(lay_);
  const int nb = lay_.nblk, k = k_;
  double* x = off<double>(lay_.off_x);
  double* b = off<double>(lay_.off_b);
  double* V = off<double>(lay_.off_V);
  double* partn = off<double>(lay_.off_partn);
  double* stat = off<double>(q.stat);
  launch_lsq(so, off<double>(q.H), off<double>(q.g), 0, k, off<double>(q.y), s_);
  launch_xupdate(so, x, off<float>(lay_.off_Z), lay_.ldz, off<double>(q.y), 0, n, s_);
  launch_dots(so, b, n, 1, b, n, partn, nb, s_);
  launch_start_cycle(so, partn, nb, nullptr, k, stat, s_);
  launch_copy_f64(so, stat + 4, off<double>(q.bn), 1, s_);
  launch_apply(T, x, 1, V, 1, b, true, s_);
  launch_dots(so, V, n, 1, V, n, partn, nb, s_);
  launch_start_cycle(so, partn, nb, off<double>(q.g), k, stat, s_);
  launch_report(so, stat, off<double>(q.bn), rep_, s_);
  RTE_HIP(hipMemcpyAsync(hrep_, rep_, size_t(zc_) * 8 * sizeof(double), hipMemcpyDeviceToHost, s_));
  RTE_HIP(hipEventRecord(ev_rep_, s_));
  phase_ = RESTART;
}

void Batch::finish_member(Member* mb, rte_status st) {
  const int z = mb->slot;
  mb->status = st;
  mb->ms = now_ms() - mb->t0;
  RTE_HIP(hipMemcpyAsync(mb->out, mb->ws + lay_.off_x, size_t(lay_.n) * 8, hipMemcpyDeviceToDevice, s_));
  RTE_HIP(hipEventCreateWithFlags(&mb->copied, hipEventDisableTiming));
  RTE_HIP(hipEventRecord(mb->copied, s_));
  hdesc_[z] = SlotDesc{};
  draining_.push_back(std::move(slot_[z]));
}

// The host's decision per slot after a boundary report, in the order of
// the single-solve driver: a non-finite right-hand side, a zero one, a
// breakdown in the last cycle, convergence of the true residual, the
// iteration limit, and stagnation (three cycles that each reduce the true
// residual by less than 0.1%).
void Batch::decide() {
  Quiet quiet;
  int cont = 0;
  for (int z = 0; z < zc_; ++z) {
    Member* mb = slot_[z].get();
    if (!mb) continue;
    const double* r = hrep_ + 8 * z;
    const double beta = r[0], bn = r[1];
    const int jj = int(r[2]);
    const bool bad = r[3] != 0.0;
    mb->iters += jj;
    if (jj > 0) ++mb->restarts;
    if (mb->bnorm < 0) {
      mb->bnorm = bn;
      if (!std::isfinite(bn)) {
        finish_member(mb, RTE_EINVAL);
        continue;
      }
      if (bn == 0.0) {
        launch_fill_f64(Slots{}, reinterpret_cast<double*>(mb->ws + lay_.off_x), 0.0, lay_.n, s_);
        mb->rel = 0;
        finish_member(mb, RTE_OK);
        continue;
      }
      mb->prev = INFINITY;
    }
    mb->rel = beta / mb->bnorm;
    if (bad || !std::isfinite(beta)) {
      finish_member(mb, RTE_EBREAKDOWN);
      continue;
    }
    if (mb->rel <= mb->o.rtol) {
      finish_member(mb, RTE_OK);
      continue;
    }
    if (mb->iters >= mb->o.max_iters) {
      finish_member(mb, RTE_ENOCONV);
      continue;
    }
    if (beta >= mb->prev * (1.0 - 1e-3)) {
      if (++mb->stall >= 3) {
        finish_member(mb, RTE_ENOCONV);
        continue;
      }
    } else {
      mb->stall = 0;
    }
    mb->prev = beta;
    SlotDesc& d = hdesc_[z];
    d.live = 1;
    d.jj = 0;
    d.bad = 0;
    d.limit = std::min(k_, mb->o.max_iters - mb->iters);
    ++cont;
  }
  upload_all();
  nlive_ = cont;
  if (cont == 0) {
    boundary();
    return;
  }
  const Small q = small_of(lay_);
  launch_scale_by(slots(0), off<double>(lay_.off_V), off<double>(q.stat) + 3, lay_.n, s_);  // v_0 = r / beta
  gcache_ = graphs_ ? step_graphs(tab_, m_, precond_, k_, key_, zc_) : nullptr;
  j_wait_ = 0;
  enqueue_step(0);
  if (k_ > 1) enqueue_step(1);
  phase_ = STEPS;
}

// Arnoldi step j for every live slot, with the second Gram-Schmidt
// correction of each new basis vector lagged into the next step:
//   the previous step left w1 = w - V h1 (once corrected, unnormalised) in
//   V[j]; the preconditioner takes v^_j = w1 / ||w1|| (stat[5]), which is
//   all flexible GMRES needs of its input (Z_j = M(v^_j) is what enters
//   A Z = V H);
//   pass 1 completes v_j = (w1 - V h2) / ||w1 - V h2|| (stat[3], h2 from the
//   previous step) in place and forms h1 = V^T w in the same read of V;
//   pass 2 forms w1 = w - V h1 with h2 = V^T w1 and ||w1||^2 in one read;
//   the finishing kernel sets column j of H (h1 + h2 over
//   ||w1 - V h2|| = sqrt(||w1||^2 - ||h2||^2)) and the Givens rotation.
// Two passes over V per step instead of three.
void Batch::step_body(int j, int zc, hipStream_t s) {
  const Slots sl{tab_, zc, 0};
  const Target T{&shape_, rel_, sl};
  const int64_t n = lay_.n;
  const int nb = lay_.nblk, k = k_;
  const Small q = small_of(lay_);
  double* V = off<double>(lay_.off_V);
  const int64_t ldv = lay_.ldv;
  double* Vj = V + size_t(j) * ldv;
  double* Vn = V + size_t(j + 1) * ldv;
  float* Zj = off<float>(lay_.off_Z) + size_t(j) * lay_.ldz;
  double* part1 = off<double>(lay_.off_part1);
  double* part2 = off<double>(lay_.off_part2);
  double* h1 = off<double>(q.h1);
  double* h2 = off<double>(q.h2);
  double* stat = off<double>(q.stat);
  if (mg_)
    precond_apply(T, *m_, kind_, Vj, Zj, off<char>(lay_.off_mg), s, stat + 5);
  else if (bj_)
    launch_block_jacobi(T, Vj, stat + 5, Zj, s);
  else
    launch_cast_f64_f32(sl, Vj, stat + 5, Zj, n, s);
  launch_apply(T, Zj, 0, Vn, 1, nullptr, false, s);
  if (j == 0)
    launch_dots(sl, V, ldv, 1, Vn, n, part1, nb, s);
  else
    launch_finish_dots(sl, V, ldv, j, h2, stat + 3, Vn, n, part1, nb, s);
  launch_reduce(sl, part1, nb, j + 1, h1, s);
  launch_updots(sl, V, ldv, j + 1, h1, Vn, n, part2, nb, s);
  launch_reduce(sl, part2, nb, j + 2, h2, s);
  launch_finish_step(sl, h1, h2, j, k, off<double>(q.H), off<double>(q.cs), off<double>(q.sn), off<double>(q.g),
                     off<double>(q.bn), stat, s);
}

namespace {

// Capture the launches of one Arnoldi step on a private stream (nothing runs
// during capture) and instantiate them as a graph.
hipGraphExec_t capture_step(Batch& b, int j, int zc) {
  thread_local hipStream_t cap = nullptr;
  if (!cap) RTE_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  prof_capturing() = true;
  hipGraph_t g = nullptr;
  RTE_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  try {
    b.step_body(j, zc, cap);
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

// Replays the step's graph (captured on first use); while the kernel-class
// timer is on, one step in `every` runs eagerly with all of its launches of
// the enabled classes timed.  The descriptors are copied back after every
// step so the host can end a cycle early.
void Batch::enqueue_step(int j) {
  const int stride = prof_stride();
  const bool sample = stride > 0 && (g_steps.fetch_add(1) % stride) == 0;
  if (!gcache_ || sample) {
    prof_force() = sample;
    prof_quiet() = !sample;
    prof_scale() = double(nlive_);
    try {
      step_body(j, zc_, s_);
    } catch (...) {
      prof_force() = false;
      prof_quiet() = false;
      prof_scale() = 1.0;
      throw;
    }
    prof_force() = false;
    prof_quiet() = false;
    prof_scale() = 1.0;
  } else {
    hipGraphExec_t& ge = (*gcache_)[j];
    if (!ge) ge = capture_step(*this, j, zc_);
    RTE_HIP(hipGraphLaunch(ge, s_));
  }
  RTE_HIP(hipMemcpyAsync(hsnap_ + size_t(j % 2) * cap_, tab_, size_t(zc_) * sizeof(SlotDesc),
                         hipMemcpyDeviceToHost, s_));
  RTE_HIP(hipEventRecord(ev_step_[j % 2], s_));
  j_enq_ = j + 1;
}

bool Batch::ready() {
  hipEvent_t e = nullptr;
  if (phase_ == RESTART) e = ev_rep_;
  else if (phase_ == STEPS) e = ev_step_[j_wait_ % 2];
  else return true;
  const hipError_t r = hipEventQuery(e);
  if (r == hipErrorNotReady) return false;
  RTE_HIP(r);
  return true;
}

void Batch::wait() {
  if (phase_ == RESTART) {
    RTE_HIP(hipEventSynchronize(ev_rep_));
  } else if (phase_ == STEPS) {
    RTE_HIP(hipEventSynchronize(ev_step_[j_wait_ % 2]));
  } else {
    for (auto& mb : draining_) RTE_HIP(hipEventSynchronize(mb->copied));
  }
}

void Batch::advance() {
  switch (phase_) {
    case IDLE:
      if (!waiting_.empty()) boundary();
      return;
    case RESTART:
      decide();
      return;
    case STEPS: {
      const int j = j_wait_;
      const SlotDesc* snap = hsnap_ + size_t(j % 2) * cap_;
      int live = 0;
      for (int z = 0; z < zc_; ++z)
        if (slot_[z] && snap[z].live) ++live;
      nlive_ = live;
      if (live == 0 || j + 1 == k_) {
        // every slot has stopped: a step j + 1 already queued finds no live
        // slot and changes nothing
        boundary();
        return;
      }
      j_wait_ = j + 1;
      if (j + 2 < k_ && j_enq_ == j + 2) enqueue_step(j + 2);
      return;
    }
  }
}

void Batch::collect(std::vector<Finished>& out) {
  for (size_t i = 0; i < draining_.size();) {
    Member* mb = draining_[i].get();
    const hipError_t r = hipEventQuery(mb->copied);
    if (r == hipErrorNotReady) {
      ++i;
      continue;
    }
    RTE_HIP(r);
    Finished f;
    f.tag = mb->tag;
    f.status = mb->status;
    f.stats.iterations = mb->iters;
    f.stats.restarts = mb->restarts;
    f.stats.converged = mb->status == RTE_OK;
    f.stats.status = mb->status;
    f.stats.rel_residual = mb->rel;
    f.stats.ms_total = mb->ms;
    out.push_back(f);
    (void)hipEventDestroy(mb->copied);
    mb->copied = nullptr;
    draining_.erase(draining_.begin() + long(i));
  }
}

void Batch::abandon(rte_status st, std::vector<Finished>& out) {
  (void)hipStreamSynchronize(s_);
  auto give = [&](std::unique_ptr<Member>& mb, rte_status code) {
    if (!mb) return;
    Finished f{};
    f.tag = mb->tag;
    f.status = code;
    f.stats.iterations = mb->iters;
    f.stats.restarts = mb->restarts;
    f.stats.status = code;
    f.stats.rel_residual = mb->rel;
    out.push_back(f);
    if (mb->copied) (void)hipEventDestroy(mb->copied);
    mb.reset();
  };
  for (auto& mb : draining_) give(mb, mb->status);
  for (auto& mb : slot_) give(mb, st);
  for (auto& mb : waiting_) give(mb, st);
  draining_.clear();
  waiting_.clear();
  std::memset(hdesc_, 0, size_t(cap_) * sizeof(SlotDesc));
  phase_ = IDLE;
  zc_ = 0;
}

}  // namespace rte

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
  // tb[l]: t_l is stored as bfloat16 (it only ever feeds convolutions, which
  // round it to bfloat16 when staging anyway).  That needs every producer and
  // consumer of t_l on the tiled 2D kernel: the level's 3x3 convolutions, the
  // restriction into it (which writes t_l) and the one out of it (which reads
  // t_l); the lift and the pointwise scaling write either form.
  // RTE_T_BF16=0 keeps every t in FP32 (for comparisons: the results are
  // bitwise the same).
  const char* tenv = std::getenv("RTE_T_BF16");
  const bool t16_ok = kind == MFMA_BF16 && op.dim == 2 && !(tenv && tenv[0] == '0');
  auto tiled3 = [&](int l) {
    return C[l] % 32 == 0 && op.level_dim(l, 0) % 8 == 0 && op.level_dim(l, 1) % 8 == 0;
  };
  std::vector<bool> tb(L, false);
  for (int l = 0; l < L; ++l)
    tb[l] = t16_ok && tiled3(l) && (l == 0 || tiled3(l - 1)) && (l == L - 1 || tiled3(l + 1));
  auto conv_same = [&](int l, const float* in, const ConvW& w, float* out, int mode) {
    ConvLaunch c{};
    int d[3];
    dims(l, d);
    conv3_setup(c, op.dim, d, 1);
    c.sl = sl;
    c.in = in; c.cin = w.cin; c.w = &w; c.out = out; c.cout = w.cout; c.mode = mode;
    c.f = f[l]; c.a = T.arr.fa[l]; c.ainv = T.arr.fainv[l];
    c.in16 = tb[l] && (mode == CONV_STORE || mode == CONV_ACCUM);  // the input is t_l
    c.t16 = tb[l] && (mode == CONV_RESID_T || mode == CONV_RESID_R);  // the output is t_l
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
      if (!tready[l]) launch_scale_fields(sl, T.arr.fainv[l], f[l], t[l], P[l] * C[l], tb[l], s);
      tready[l] = false;
      conv_same(l, t[l], B, u[l], CONV_STORE);
      uz[l] = false;
    } else {
      conv_same(l, u[l], m.A[l], t[l], CONV_RESID_T);
      conv_same(l, t[l], B, u[l], CONV_ACCUM);
    }
  };

  const bool want0 = first_steps(0) > 0;
  launch_lift(T, m, v, vscale, f[0], want0 ? T.arr.fainv[0] : nullptr, want0 ? t[0] : nullptr, tb[0], s);
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
    c.in16 = tb[l] && !uz[l];       // the input is t_l (else f_l)
    c.t16 = tb[l + 1] && want;      // out2 is t_{l+1}
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
  return align256(size_t(capacity) * sizeof(SlotDesc)) + align256(size_t(capacity) * sizeof(SlotInit)) +
         align256(size_t(capacity) * sizeof(SlotEmit));
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

struct GraphEntry {
  std::vector<hipGraphExec_t> g = std::vector<hipGraphExec_t>(5, nullptr);  // register budgets 4, 8, 16, 32, 64
  uint64_t used = 0;
};
std::mutex g_graph_mu;
std::map<GraphKey, std::unique_ptr<GraphEntry>>& graph_map() {
  static auto* m = new std::map<GraphKey, std::unique_ptr<GraphEntry>>();
  return *m;
}
std::map<const void*, int>& held_tables() {
  static auto* m = new std::map<const void*, int>();
  return *m;
}
uint64_t g_graph_clock = 0;
// keys kept beyond the ones of tables in use
constexpr size_t GRAPH_CACHE_KEYS = 32;

void destroy_entry(GraphEntry& e) {
  for (hipGraphExec_t x : e.g)
    if (x) (void)hipGraphExecDestroy(x);
}

// with g_graph_mu held: evict least recently used keys of tables not in use
void trim_graphs() {
  auto& mp = graph_map();
  auto& held = held_tables();
  while (mp.size() > GRAPH_CACHE_KEYS) {
    auto victim = mp.end();
    for (auto it = mp.begin(); it != mp.end(); ++it)
      if (!held.count(it->first.tab) && (victim == mp.end() || it->second->used < victim->second->used))
        victim = it;
    if (victim == mp.end()) return;
    destroy_entry(*victim->second);
    mp.erase(victim);
  }
}

std::atomic<int64_t> g_steps{0};  // ticks enqueued by every batch (timer sampling)

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

std::vector<hipGraphExec_t>* step_graphs(const void* tab, const Model* m, int precond, int k,
                                         const std::vector<int64_t>& shape, int zc) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto& slot = graph_map()[GraphKey{tab, m, precond, k, zc, shape}];
  if (!slot) slot.reset(new GraphEntry());
  slot->used = ++g_graph_clock;
  std::vector<hipGraphExec_t>* r = &slot->g;
  trim_graphs();  // the caller's table is held, so its entry stays
  return r;
}

void step_graphs_hold(const void* tab) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  ++held_tables()[tab];
}

void step_graphs_release(const void* tab) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto& held = held_tables();
  auto it = held.find(tab);
  if (it != held.end() && --it->second == 0) held.erase(it);
  trim_graphs();
}

void drop_step_graphs(const Model* m) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto& mp = graph_map();
  for (auto it = mp.begin(); it != mp.end();) {
    if (it->first.m == m) {
      destroy_entry(*it->second);
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
  if (op.scheme == RTE_SCHEME_TFPS)
    RTE_REQUIRE(o->precond == RTE_PC_NONE, RTE_EINVAL,
                "the TFPS operator is solved without a preconditioner (MgNet and Block-Jacobi act on the upwind scheme)");
  if (o->precond == RTE_PC_BLOCK_JACOBI)
    RTE_REQUIRE(op.ndir <= RTE_BJ_MAX_DIRS, RTE_EINVAL, "Block-Jacobi supports up to 112 directions");
  if (o->precond == RTE_PC_MGNET_BF16 || o->precond == RTE_PC_MGNET_FP32) {
    RTE_REQUIRE(m != nullptr, RTE_EINVAL, "MgNet preconditioning needs a model");
    RTE_REQUIRE(op.model == m, RTE_EINVAL, "operator was not built with this model (CoeffNet fields missing)");
  }
}

Batch::Batch(const Operator& shape, const Model* m, int k, int precond, int capacity, char* tables,
             hipStream_t s)
    : shape_(shape.geometry()), key_(shape.shape_key()), m_(m), k_(k), precond_(precond), cap_(capacity), s_(s) {
  RTE_REQUIRE(capacity >= 1 && capacity <= 64, RTE_EINVAL, "batch capacity must be in [1, 64]");
  RTE_REQUIRE(tables != nullptr && (reinterpret_cast<uintptr_t>(tables) & 255) == 0, RTE_EINVAL,
              "batch tables must be 256-byte aligned");
  mg_ = precond == RTE_PC_MGNET_BF16 || precond == RTE_PC_MGNET_FP32;
  bj_ = precond == RTE_PC_BLOCK_JACOBI;
  kind_ = precond == RTE_PC_MGNET_FP32 ? MFMA_F32 : MFMA_BF16;
  lay_ = solve_layout(shape, m, k, mg_);
  rel_ = shape.relative();
  tab_ = reinterpret_cast<SlotDesc*>(tables);
  dinit_ = reinterpret_cast<SlotInit*>(tables + align256(size_t(capacity) * sizeof(SlotDesc)));
  demit_ = reinterpret_cast<SlotEmit*>(reinterpret_cast<char*>(dinit_) + align256(size_t(capacity) * sizeof(SlotInit)));
  if (mg_) const_cast<Model*>(m)->ensure_on_device();
  const char* env = std::getenv("RTE_GRAPHS");
  graphs_ = !(env && env[0] == '0');
  slot_.resize(size_t(capacity));
  RTE_HIP(hipHostMalloc(reinterpret_cast<void**>(&hdesc_), size_t(capacity) * sizeof(SlotDesc),
                        hipHostMallocDefault));
  RTE_HIP(hipHostMalloc(reinterpret_cast<void**>(&hsnap_), 2 * size_t(capacity) * sizeof(SlotDesc),
                        hipHostMallocDefault));
  RTE_HIP(hipHostMalloc(reinterpret_cast<void**>(&hinit_), 2 * size_t(capacity) * sizeof(SlotInit),
                        hipHostMallocDefault));
  RTE_HIP(hipHostMalloc(reinterpret_cast<void**>(&hemit_), 2 * size_t(capacity) * sizeof(SlotEmit),
                        hipHostMallocDefault));
  std::memset(hdesc_, 0, size_t(capacity) * sizeof(SlotDesc));
  std::memset(hsnap_, 0, 2 * size_t(capacity) * sizeof(SlotDesc));
  std::memset(hinit_, 0, 2 * size_t(capacity) * sizeof(SlotInit));
  std::memset(hemit_, 0, 2 * size_t(capacity) * sizeof(SlotEmit));
  for (auto& e : ev_tick_) RTE_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  upload_all();
  step_graphs_hold(tab_);
}

Batch::~Batch() {
  (void)hipStreamSynchronize(s_);
  step_graphs_release(tab_);
  waiting_.clear();
  draining_.clear();
  slot_.clear();
  for (auto& e : ev_tick_)
    if (e) (void)hipEventDestroy(e);
  if (hdesc_) (void)hipHostFree(hdesc_);
  if (hsnap_) (void)hipHostFree(hsnap_);
  if (hinit_) (void)hipHostFree(hinit_);
  if (hemit_) (void)hipHostFree(hemit_);
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

bool Batch::idle() const {
  return t_done_ == t_enq_ && members() == 0 && draining_.empty();
}

void Batch::upload_all() {
  RTE_HIP(hipMemcpyAsync(tab_, hdesc_, size_t(cap_) * sizeof(SlotDesc), hipMemcpyHostToDevice, s_));
}

namespace {
// The admission and result launches read x0 and b and write the output in
// a kernel: each must be device memory (a host address would fault there).
void require_device(const void* p, const char* what) {
  hipPointerAttribute_t a{};
  const hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) (void)hipGetLastError();  // clear the sticky query error
  RTE_REQUIRE(e == hipSuccess && (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged ||
                                  a.type == hipMemoryTypeUnified || a.isManaged),
              RTE_EINVAL, std::string(what) + " must be device memory");
}
}  // namespace

void Batch::add(void* tag, const Operator& op, const rte_solve_opts& o, char* ws, double* out, double t_start) {
  RTE_REQUIRE(o.restart == k_ && o.precond == precond_ && op.shape_key() == key_ && (!mg_ || op.model == m_),
              RTE_EINVAL, "solve does not match the batch");
  RTE_REQUIRE(!full(), RTE_EINVAL, "batch is full");
  RTE_REQUIRE(ws && out && (reinterpret_cast<uintptr_t>(ws) & 255) == 0, RTE_EINVAL,
              "bad workspace or output");
  require_device(out, "the output");
  if (o.x0) require_device(o.x0, "x0");
  if (o.b) require_device(o.b, "b");
  std::unique_ptr<Member> mb(new Member());
  mb->tag = tag;
  mb->op = &op;
  mb->o = o;
  mb->ws = ws;
  mb->out = out;
  mb->t0 = t_start;
  waiting_.push_back(std::move(mb));
}

namespace {
struct Quiet {
  Quiet() { prof_quiet() = true; }
  ~Quiet() { prof_quiet() = false; }
};
int pow2_at_least(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}
// register budget index of the dot kernels for steps j <= jmax: 4, 8, 16, 32, 64
// (the first steps of a batch take the 4-vector kernels, without the
// clamped reloads of a wider budget)
int budget_index(int jmax) {
  const int nv = jmax + 1;
  return nv <= 4 ? 0 : nv <= 8 ? 1 : nv <= 16 ? 2 : nv <= 32 ? 3 : 4;
}
}  // namespace

// A waiting solve takes slot z: staged for the tick's admission launch,
// which sets x = x0 (or 0), copies the right-hand side into the workspace
// and writes the descriptor: the slot waits at a cycle edge with no steps
// taken, so the boundary launches that follow form r = b - L x and decide
// (normally: a first cycle).
void Batch::admit(int z, SlotInit& in) {
  std::unique_ptr<Member> mb = std::move(waiting_.front());
  waiting_.erase(waiting_.begin());
  SlotDesc d{};
  d.ws = reinterpret_cast<uint64_t>(mb->ws);
  d.op = reinterpret_cast<uint64_t>(mb->op->block);
  d.occupied = 1;
  d.edge = 1;
  d.rtol = mb->o.rtol;
  d.max_iters = mb->o.max_iters;
  d.bnorm = -1.0;
  in.d = d;
  in.x0 = reinterpret_cast<uint64_t>(mb->o.x0);
  in.b = reinterpret_cast<uint64_t>(mb->o.b ? static_cast<const double*>(mb->o.b) : mb->op->a.b64);
  in.admit = 1;
  mb->slot = z;
  mb->since = t_enq_;
  mb->bnd_tick = t_enq_;
  slot_[z] = std::move(mb);
}

// Cycle boundary of every slot at the edge: combine the ended cycle's steps
// into x (x += Z y), form the FP64 true residual r = b - L x as V[0], its
// norm and ||b||, and take the restart-or-finish decision on the device.
void Batch::boundary_launches(int zc) {
  Quiet quiet;
  const Slots so{tab_, zc, GATE_EDGE};
  const Target T{shape_.get(), rel_, so};
  const Small q = small_of(lay_);
  const int64_t n = lay_.n;
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
  launch_operator(T, x, 1, V, 1, b, true, s_);
  launch_dots(so, V, n, 1, V, n, partn, nb, s_);
  launch_start_cycle(so, partn, nb, off<double>(q.g), k, stat, s_);
  launch_decide(so, stat, off<double>(q.bn), k, s_);
}

// Arnoldi step j of every live slot, each at its own j, with the second
// Gram-Schmidt correction of each new basis vector lagged into the next
// step:
//   the previous step left w1 = w - V h1 (once corrected, unnormalised) in
//   V[j] (at j = 0: the residual r); the preconditioner takes
//   v^_j = w1 / ||w1|| (r / beta; scale stat[5]), which is all flexible
//   GMRES needs of its input (Z_j = M(v^_j) is what enters A Z = V H);
//   pass 1 completes v_j = (w1 - V h2) / ||w1 - V h2|| (stat[3], h2 from the
//   previous step; at j = 0, r / beta) in place and forms h1 = V^T w in the
//   same read of V;
//   pass 2 forms w1 = w - V h1 with h2 = V^T w1 and ||w1||^2 in one read;
//   the finishing kernel sets column j of H (h1 + h2 over
//   ||w1 - V h2|| = sqrt(||w1||^2 - ||h2||^2)) and the Givens rotation.
// Two passes over V per step instead of three.  The step-indexed operands
// (V_j, Z_j, V_{j+1}) are passed at j = 0 and moved by each slot's jj.
void Batch::step_body(int jmax, int zc, hipStream_t s) {
  const int64_t n = lay_.n;
  const int nb = lay_.nblk, k = k_;
  const Small q = small_of(lay_);
  double* V = off<double>(lay_.off_V);
  float* Z = off<float>(lay_.off_Z);
  const int64_t ldv = lay_.ldv, ldz = lay_.ldz;
  const Slots sl{tab_, zc, GATE_LIVE};
  const Slots vz{tab_, zc, GATE_LIVE, ldv * 8, ldz * 4};  // V_j in, Z_j out
  const Slots zv{tab_, zc, GATE_LIVE, ldz * 4, ldv * 8};  // Z_j in, V_{j+1} out
  const Target Tvz{shape_.get(), rel_, vz};
  const Target Tzv{shape_.get(), rel_, zv};
  double* part1 = off<double>(lay_.off_part1);
  double* part2 = off<double>(lay_.off_part2);
  double* h1 = off<double>(q.h1);
  double* h2 = off<double>(q.h2);
  double* stat = off<double>(q.stat);
  if (mg_)
    precond_apply(Tvz, *m_, kind_, V, Z, off<char>(lay_.off_mg), s, stat + 5);
  else if (bj_)
    launch_block_jacobi(Tvz, V, stat + 5, Z, s);
  else
    launch_cast_f64_f32(vz, V, stat + 5, Z, n, s);
  launch_operator(Tzv, Z, 0, V + ldv, 1, nullptr, false, s);
  launch_finish_dots(sl, V, ldv, jmax, h2, stat + 3, n, part1, nb, s);
  launch_reduce(sl, part1, nb, jmax + 1, h1, s);
  launch_updots(sl, V, ldv, jmax, h1, n, part2, nb, s);
  launch_reduce(sl, part2, nb, jmax + 2, h2, s);
  launch_finish_step(sl, h1, h2, k, jmax, off<double>(q.H), off<double>(q.cs), off<double>(q.sn),
                     off<double>(q.g), off<double>(q.bn), stat, s);
}

namespace {

// Capture the launches of one Arnoldi step on a private stream (nothing runs
// during capture) and instantiate them as a graph.
hipGraphExec_t capture_step(Batch& b, int jmax, int zc) {
  thread_local hipStream_t cap = nullptr;
  if (!cap) RTE_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  prof_capturing() = true;
  hipGraph_t g = nullptr;
  RTE_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  try {
    b.step_body(jmax, zc, cap);
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

// One tick: admissions into free slots, the boundary launches when a slot
// waits at an edge, the step (a graph per register budget and slot count;
// while the kernel-class timer is on, one tick in `every` runs the step
// eagerly with its launches timed), and the copy of the table.
void Batch::enqueue_tick() {
  const int64_t t = t_enq_;
  SlotInit* init = hinit_ + size_t(t % 2) * cap_;
  bool bnd = false;
  for (int z = 0; z < cap_ && !waiting_.empty(); ++z)
    if (!slot_[z]) {
      if (!bnd) std::memset(init, 0, size_t(cap_) * sizeof(SlotInit));
      admit(z, init[z]);
      bnd = true;
    }
  const bool admitted = bnd;
  int hi = 0;
  for (int z = 0; z < cap_; ++z)
    if (slot_[z]) {
      hi = z + 1;
      if (slot_[z]->edge_pending) bnd = true;
    }
  // the launches cover a power-of-two prefix of the slots that only grows
  // while the batch is busy, so few step graphs exist per batch
  zc_ = std::max(zc_, std::min(cap_, pow2_at_least(std::max(hi, 1))));
  const int zc = zc_;
  if (admitted) {
    Quiet quiet;
    RTE_HIP(hipMemcpyAsync(dinit_, init, size_t(zc) * sizeof(SlotInit), hipMemcpyHostToDevice, s_));
    launch_admit(tab_, dinit_, zc, lay_.n, lay_.off_x, lay_.off_b, s_);
  }
  if (bnd) {
    boundary_launches(zc);
    for (int z = 0; z < cap_; ++z)
      if (slot_[z]) {
        slot_[z]->bnd_tick = t;
        slot_[z]->edge_pending = false;
      }
  }
  // a slot live at the last table read had jj <= snap_jmax_ then and takes
  // one step per tick since; a slot restarted since has taken fewer
  const int lag = int(t - 1 - snap_tick_);
  const int jtrue = std::min(k_ - 1, snap_jmax_ + lag);
  const int bi = budget_index(jtrue);
  const int jmax = (4 << bi) - 1;
  const int stride = prof_stride();
  const bool sample = stride > 0 && (g_steps.fetch_add(1) % stride) == 0;
  if (!graphs_ || sample) {
    std::shared_ptr<double> sc;
    if (sample) {
      sc = std::make_shared<double>(-1.0);
      tick_scale_[t % 2] = sc;
    }
    prof_force() = sample;
    prof_quiet() = !sample;
    prof_scale() = sc;
    try {
      step_body(jmax, zc, s_);
    } catch (...) {
      prof_force() = false;
      prof_quiet() = false;
      prof_scale().reset();
      throw;
    }
    prof_force() = false;
    prof_quiet() = false;
    prof_scale().reset();
  } else {
    std::vector<hipGraphExec_t>* gc = step_graphs(tab_, m_, precond_, k_, key_, zc);
    hipGraphExec_t& ge = (*gc)[size_t(bi)];
    if (!ge) ge = capture_step(*this, jmax, zc);
    RTE_HIP(hipGraphLaunch(ge, s_));
  }
  RTE_HIP(hipMemcpyAsync(hsnap_ + size_t(t % 2) * cap_, tab_, size_t(zc) * sizeof(SlotDesc),
                         hipMemcpyDeviceToHost, s_));
  RTE_HIP(hipEventRecord(ev_tick_[t % 2], s_));
  tick_zc_[t % 2] = zc;
  t_enq_ = t + 1;
}

bool Batch::ready() {
  if (t_done_ == t_enq_) return true;
  const hipError_t r = hipEventQuery(ev_tick_[t_done_ % 2]);
  if (r == hipErrorNotReady) return false;
  RTE_HIP(r);
  return true;
}

void Batch::wait() {
  if (t_done_ < t_enq_) {
    RTE_HIP(hipEventSynchronize(ev_tick_[t_done_ % 2]));
  } else {
    for (auto& mb : draining_) RTE_HIP(hipEventSynchronize(mb->copied->e));
  }
}

// A finished solve: its x (or zeros, for b = 0) goes to the caller's buffer
// by the emit launch queued behind the ticks already in flight, which leave
// the slot untouched.
void Batch::finish_member(int z, const SlotDesc& d, SlotEmit& em) {
  std::unique_ptr<Member>& mb = slot_[z];
  mb->iters = d.iters;
  mb->restarts = d.restarts;
  mb->rel = d.rel;
  mb->status = rte_status(d.code);
  mb->ms = now_ms() - mb->t0;
  em.out = reinterpret_cast<uint64_t>(mb->out);
  em.x = reinterpret_cast<uint64_t>(mb->ws + lay_.off_x);
  em.mode = d.done == 2 ? 2 : 1;
  draining_.push_back(std::move(mb));
}

// Reads the table copy of tick t: finished solves (emitted together, with
// one completion event), slots waiting at an edge, the largest step of a
// live slot, and how many slots stepped (the work multiplier of a timed
// tick).
void Batch::process(int64_t t) {
  const SlotDesc* snap = hsnap_ + size_t(t % 2) * cap_;
  SlotEmit* em = hemit_ + size_t(t % 2) * cap_;
  const int zc = tick_zc_[t % 2];
  const size_t first_out = draining_.size();
  int jm = 0, stepped = 0;
  for (int z = 0; z < zc; ++z) {
    Member* mb = slot_[z].get();
    if (!mb || mb->since > t) continue;
    const SlotDesc& d = snap[z];
    if (d.steps > mb->steps_seen) {
      ++stepped;
      mb->steps_seen = d.steps;
    }
    if (d.done) {
      if (draining_.size() == first_out) std::memset(em, 0, size_t(zc) * sizeof(SlotEmit));
      finish_member(z, d, em[z]);
      continue;
    }
    if (d.live) jm = std::max(jm, int(d.jj));
    // an edge already covered by a boundary queued after tick t is not new
    if (d.edge && mb->bnd_tick <= t) mb->edge_pending = true;
  }
  if (draining_.size() > first_out) {
    Quiet quiet;
    RTE_HIP(hipMemcpyAsync(demit_, em, size_t(zc) * sizeof(SlotEmit), hipMemcpyHostToDevice, s_));
    launch_emit(demit_, zc, lay_.n, s_);
    std::shared_ptr<Event> ev(new Event());
    RTE_HIP(hipEventCreateWithFlags(&ev->e, hipEventDisableTiming));
    RTE_HIP(hipEventRecord(ev->e, s_));
    for (size_t i = first_out; i < draining_.size(); ++i) draining_[i]->copied = ev;
  }
  snap_tick_ = t;
  snap_jmax_ = jm;
  if (tick_scale_[t % 2]) {
    *tick_scale_[t % 2] = double(stepped);
    tick_scale_[t % 2].reset();
  }
  t_done_ = t + 1;
}

void Batch::fill() {
  while (t_enq_ - t_done_ < 2) {
    bool work = !waiting_.empty();
    for (auto& mb : slot_)
      if (mb) work = true;
    if (!work) {
      if (t_enq_ == t_done_) zc_ = 0;  // nothing in flight or held: start small again
      return;
    }
    enqueue_tick();
  }
}

void Batch::advance() {
  if (t_done_ < t_enq_) process(t_done_);
  fill();
}

void Batch::collect(std::vector<Finished>& out) {
  for (size_t i = 0; i < draining_.size();) {
    Member* mb = draining_[i].get();
    const hipError_t r = hipEventQuery(mb->copied->e);
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
    mb.reset();
  };
  for (auto& mb : draining_) give(mb, mb->status);
  for (auto& mb : slot_) give(mb, st);
  for (auto& mb : waiting_) give(mb, st);
  draining_.clear();
  waiting_.clear();
  for (auto& sc : tick_scale_) {
    if (sc) *sc = 0.0;
    sc.reset();
  }
  t_done_ = t_enq_ = 0;
  snap_tick_ = -1;
  snap_jmax_ = 0;
  zc_ = 0;
  // every slot off before the table is used again
  std::memset(hdesc_, 0, size_t(cap_) * sizeof(SlotDesc));
  try {
    upload_all();
    RTE_HIP(hipStreamSynchronize(s_));
  } catch (...) {
  }
}

}  // namespace rte

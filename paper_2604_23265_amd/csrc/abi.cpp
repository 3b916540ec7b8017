// extern "C" entry points of librte: argument checks, error mapping and the
// kernel-class event timer.
#include <chrono>
#include <cstring>
#include <memory>

#include "common.h"

namespace rte {

Operator* build_operator(const rte_geometry* g, const rte_medium* md, const Model* model, hipStream_t stream);
Model* parse_mgn1(const void* blob, size_t bytes);

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

void fail(rte_status code, const std::string& msg) { throw Error(code, msg); }

// ------------------------------------------------------------- profiler ---
namespace {
constexpr size_t kProfEventReserve = 8192;
struct Prof {
  std::mutex mu;
  int every[RTE_K_COUNT] = {};
  int64_t seen[RTE_K_COUNT] = {};
  struct Rec {
    hipEvent_t e0, e1;
    double work, bytes;
    std::shared_ptr<double> scale;  // null: 1; negative: not known yet
    int key;
  };
  std::vector<Rec> pending[RTE_K_COUNT];
  std::vector<hipEvent_t> pool;
  double ms[RTE_K_COUNT] = {};
  double work[RTE_K_COUNT] = {};
  double bytes[RTE_K_COUNT] = {};
  int64_t count[RTE_K_COUNT] = {};
  // the same sums split by the launch's key (RTE_PROF_KEYS of them per class)
  double kms[RTE_K_COUNT][RTE_PROF_KEYS] = {};
  double kwork[RTE_K_COUNT][RTE_PROF_KEYS] = {};
  double kbytes[RTE_K_COUNT][RTE_PROF_KEYS] = {};
  int64_t kcount[RTE_K_COUNT][RTE_PROF_KEYS] = {};
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    RTE_HIP(hipEventCreate(&e));
    return e;
  }
  // folds in the records whose work multiplier is known; the others stay
  void drain(int c) {
    std::vector<Rec> keep;
    for (auto& pr : pending[c]) {
      if (pr.scale && *pr.scale < 0) {
        keep.push_back(pr);
        continue;
      }
      RTE_HIP(hipEventSynchronize(pr.e1));
      float t = 0;
      RTE_HIP(hipEventElapsedTime(&t, pr.e0, pr.e1));
      const double sc = pr.scale ? *pr.scale : 1.0;
      ms[c] += t;
      work[c] += pr.work * sc;
      bytes[c] += pr.bytes * sc;
      count[c] += 1;
      const int k = pr.key;
      kms[c][k] += t;
      kwork[c][k] += pr.work * sc;
      kbytes[c][k] += pr.bytes * sc;
      kcount[c][k] += 1;
      pool.push_back(pr.e0);
      pool.push_back(pr.e1);
    }
    pending[c].swap(keep);
  }
};
Prof& prof() {
  static Prof* p = new Prof();  // never destroyed: events outlive static teardown order
  return *p;
}
}  // namespace

bool& prof_capturing() {
  thread_local bool v = false;
  return v;
}

bool& prof_force() {
  thread_local bool v = false;
  return v;
}

bool& prof_quiet() {
  thread_local bool v = false;
  return v;
}

std::shared_ptr<double>& prof_scale() {
  thread_local std::shared_ptr<double> v;
  return v;
}

int prof_stride() {
  Prof& P = prof();
  int s = 0;
  for (int c = 0; c < RTE_K_COUNT; ++c)
    if (P.every[c] > 0 && (s == 0 || P.every[c] < s)) s = P.every[c];
  return s;
}

ProfScope::ProfScope(int c, hipStream_t st, bool ext_launch) : cls(c), s(st), ext(ext_launch) {
  Prof& P = prof();
  if (P.every[c] <= 0 || prof_capturing() || (prof_quiet() && !prof_force())) return;
  std::lock_guard<std::mutex> lk(P.mu);
  if (P.every[c] <= 0) return;
  if (!prof_force() && (P.seen[c]++ % P.every[c]) != 0) return;
  e0 = P.get();
  e1 = P.get();
  if (!ext) RTE_HIP(hipEventRecord(e0, s));
}

ProfScope::~ProfScope() {
  if (!e0) return;
  Prof& P = prof();
  std::lock_guard<std::mutex> lk(P.mu);
  try {
    if (!ext) (void)hipEventRecord(e1, s);
    const int k = key >= 0 && key < RTE_PROF_KEYS ? key : 0;
    P.pending[cls].push_back({e0, e1, work, bytes < 0 ? work : bytes, prof_scale(), k});
    if (P.pending[cls].size() >= 65536) P.drain(cls);
  } catch (...) {
  }
}

}  // namespace rte

using namespace rte;

namespace {

template <class F>
rte_status guarded(F&& f) {
  try {
    f();
    set_last_error("");
    return RTE_OK;
  } catch (const Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return RTE_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return RTE_EDEVICE;
  }
}

hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

// Whether the FP64 ranges [a, a + na) and [b, b + nb) share memory.
bool overlap(const double* a, int64_t na, const double* b, int64_t nb) {
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
  return a0 < b0 + uintptr_t(nb) * 8 && b0 < a0 + uintptr_t(na) * 8;
}

}  // namespace


extern "C" {

const char* rte_last_error(void) { return g_last_error.c_str(); }

rte_status mgnet_load(const void* blob, size_t bytes, mgnet_model** out) {
  return guarded([&] {
    RTE_REQUIRE(out != nullptr, RTE_EINVAL, "mgnet_load: null output");
    std::unique_ptr<Model> m(parse_mgn1(blob, bytes));
    auto* h = new mgnet_model();
    h->m = std::move(m);
    *out = h;
  });
}

rte_status mgnet_free(mgnet_model* model) {
  return guarded([&] {
    if (model) drop_step_graphs(model->m.get());
    delete model;
  });
}

rte_status mgnet_describe(const mgnet_model* h, int* d) {
  return guarded([&] {
    RTE_REQUIRE(h && d, RTE_EINVAL, "mgnet_describe: null argument");
    const Model& m = *h->m;
    int v[8] = {m.dim, m.ndir, m.c0, m.levels, m.nu_pre, m.nu_post, m.nu_coarse, m.coef_ch};
    std::memcpy(d, v, sizeof(v));
  });
}

rte_status rte_build_operator(const rte_geometry* geom, const rte_medium* med, const mgnet_model* model,
                              void* stream, rte_operator** out) {
  return guarded([&] {
    RTE_REQUIRE(out != nullptr, RTE_EINVAL, "rte_build_operator: null output");
    std::unique_ptr<Operator> op(build_operator(geom, med, model ? model->m.get() : nullptr, S(stream)));
    auto* h = new rte_operator();
    h->op = std::move(op);
    *out = h;
  });
}

rte_status rte_operator_free(rte_operator* op) {
  return guarded([&] {
    delete op;
  });
}

rte_status rte_operator_get_info(const rte_operator* h, rte_operator_info* info) {
  return guarded([&] {
    RTE_REQUIRE(h && info, RTE_EINVAL, "rte_operator_get_info: null argument");
    const Operator& o = *h->op;
    info->dim = o.dim; info->nx = o.nx; info->ny = o.ny; info->nz = o.nz; info->ndir = o.ndir;
    info->kernel = o.kernel; info->cells = o.cells; info->n = o.n; info->h = o.h; info->g = o.g;
    info->has_fields = o.model != nullptr;
    info->scheme = o.scheme;
    info->nbasis = o.scheme == RTE_SCHEME_TFPS ? int64_t(o.nbasis) : 0;
  });
}

rte_status rte_operator_copy_array(const rte_operator* h, int which, int level, void* dst, size_t bytes,
                                   void* stream) {
  return guarded([&] {
    RTE_REQUIRE(h && dst, RTE_EINVAL, "rte_operator_copy_array: null argument");
    const Operator& o = *h->op;
    const void* src = nullptr;
    size_t need = 0;
    DevArena tmp;
    switch (which) {
      case RTE_ARR_RHS: src = o.a.b64; need = size_t(o.n) * 8; break;
      case RTE_ARR_SCATTER: src = o.a.S64; need = size_t(o.ndir) * o.ndir * 8; break;
      case RTE_ARR_SIGMA: {
        need = size_t(o.cells) * 16;
        RTE_REQUIRE(bytes == need, RTE_EINVAL, "rte_operator_copy_array: wrong size");
        RTE_HIP(hipMemcpyAsync(dst, o.a.sT64, size_t(o.cells) * 8, hipMemcpyDeviceToDevice, S(stream)));
        RTE_HIP(hipMemcpyAsync(static_cast<char*>(dst) + size_t(o.cells) * 8, o.a.sA64, size_t(o.cells) * 8,
                               hipMemcpyDeviceToDevice, S(stream)));
        return;
      }
      case RTE_ARR_FIELD_A:
      case RTE_ARR_FIELD_AINV: {
        RTE_REQUIRE(o.model != nullptr, RTE_EINVAL, "operator has no CoeffNet fields");
        RTE_REQUIRE(level >= 0 && level < o.model->levels, RTE_EINVAL, "level out of range");
        src = which == RTE_ARR_FIELD_A ? o.a.fa[level] : o.a.fainv[level];
        need = size_t(o.level_cells(level)) * (o.model->c0 << level) * 4;
        break;
      }
      default: fail(RTE_EINVAL, "unknown array");
    }
    RTE_REQUIRE(bytes == need, RTE_EINVAL, "rte_operator_copy_array: wrong size");
    RTE_HIP(hipMemcpyAsync(dst, src, need, hipMemcpyDeviceToDevice, S(stream)));
  });
}

rte_status rte_apply(const rte_operator* h, const void* x, void* y, int precision, void* stream) {
  return guarded([&] {
    RTE_REQUIRE(h && x && y, RTE_EINVAL, "rte_apply: null argument");
    RTE_REQUIRE(x != y, RTE_EINVAL, "rte_apply: x and y must not alias");
    RTE_REQUIRE(precision == RTE_FP32 || precision == RTE_FP64, RTE_EINVAL, "rte_apply: bad precision");
    const int t = precision == RTE_FP64 ? 1 : 0;
    launch_operator(Target::single(*h->op), x, t, y, t, nullptr, precision == RTE_FP64, S(stream));
  });
}

rte_status rte_residual(const rte_operator* h, const double* x, double* r, void* stream) {
  return guarded([&] {
    RTE_REQUIRE(h && x && r, RTE_EINVAL, "rte_residual: null argument");
    RTE_REQUIRE(static_cast<const void*>(x) != static_cast<const void*>(r), RTE_EINVAL,
                "rte_residual: x and r must not alias");
    launch_operator(Target::single(*h->op), x, 1, r, 1, h->op->a.b64, true, S(stream));
  });
}

rte_status rte_cell_values(const rte_operator* h, const double* x, double* psi, void* stream) {
  return guarded([&] {
    RTE_REQUIRE(h && x && psi, RTE_EINVAL, "rte_cell_values: null argument");
    RTE_REQUIRE(static_cast<const void*>(x) != static_cast<const void*>(psi), RTE_EINVAL,
                "rte_cell_values: x and psi must not alias");
    const Operator& o = *h->op;
    if (o.scheme == RTE_SCHEME_TFPS)
      launch_tfps_centres(Target::single(o), x, psi, S(stream));
    else
      RTE_HIP(hipMemcpyAsync(psi, x, size_t(o.n) * 8, hipMemcpyDeviceToDevice, S(stream)));
  });
}

rte_status rte_atfps_build(const rte_operator* h, double delta, rte_atfps** out) {
  return guarded([&] {
    RTE_REQUIRE(h && out, RTE_EINVAL, "rte_atfps_build: null argument");
    std::unique_ptr<rte_atfps> a(new rte_atfps());
    a->op = h->op.get();
    a->host = atfps_build_host(*h->op, delta);
    RTE_HIP(hipGetDevice(&a->device));
    auto up = [&](const HostCsr& m) {
      DevCsr d;
      d.nrows = m.nrows;
      d.ncols = m.ncols;
      d.ptr = a->mem.upload(m.ptr);
      d.col = a->mem.upload(m.col);
      d.val = a->mem.upload(m.val);
      return d;
    };
    a->A = up(a->host.A);
    a->R = up(a->host.R);
    a->M = up(a->host.M);
    a->b = a->mem.upload(a->host.b);
    a->r0 = a->mem.upload(a->host.r0);
    a->c0 = a->mem.upload(a->host.c0);
    a->part = a->mem.upload(std::vector<double>(size_t(kNorm2Parts), 0.0));
    *out = a.release();
  });
}

rte_status rte_atfps_free(rte_atfps* a) {
  return guarded([&] { delete a; });
}

rte_status rte_atfps_get_info(const rte_atfps* a, int64_t* n_kept, int64_t* n_rows, int64_t* nnz) {
  return guarded([&] {
    RTE_REQUIRE(a, RTE_EINVAL, "rte_atfps_get_info: null handle");
    if (n_kept) *n_kept = a->host.n_kept;
    if (n_rows) *n_rows = a->host.n_rows;
    if (nnz) *nnz = int64_t(a->host.A.val.size());
  });
}

rte_status rte_atfps_residual(const rte_atfps* a, const double* alpha, double* r, void* stream) {
  return guarded([&] {
    RTE_REQUIRE(a && ((alpha && r) || a->host.n_kept == 0), RTE_EINVAL, "rte_atfps_residual: null argument");
    RTE_REQUIRE(!overlap(alpha, a->host.n_kept, r, a->host.n_rows), RTE_EINVAL, "rte_atfps_residual: alpha and r overlap");
    launch_csr(a->A, alpha, a->b, true, r, S(stream));
  });
}

rte_status rte_atfps_reconstruct(const rte_atfps* a, const double* alpha, double* coef, void* stream) {
  return guarded([&] {
    RTE_REQUIRE(a && coef && (alpha || a->host.n_kept == 0), RTE_EINVAL, "rte_atfps_reconstruct: null argument");
    RTE_REQUIRE(!overlap(alpha, a->host.n_kept, coef, a->host.n_full), RTE_EINVAL,
                "rte_atfps_reconstruct: alpha and coef overlap");
    launch_csr(a->R, alpha, a->r0, false, coef, S(stream));
  });
}

rte_status rte_atfps_filtered_loss(const rte_atfps* a, const double* psi, double* rho, double* loss, void* stream) {
  return guarded([&] {
    RTE_REQUIRE(a && psi && loss && (rho || a->host.n_rows == 0), RTE_EINVAL,
                "rte_atfps_filtered_loss: null argument");
    RTE_REQUIRE(!overlap(psi, int64_t(a->host.ndir) * a->host.cells, rho, a->host.n_rows), RTE_EINVAL,
                "rte_atfps_filtered_loss: psi and rho overlap");
    launch_csr(a->M, psi, a->c0, true, rho, S(stream));
    launch_norm2(rho, a->host.n_rows, a->part, loss, S(stream));
  });
}

rte_status rte_precond_workspace_bytes(const rte_operator* h, const mgnet_model* model, size_t* bytes) {
  return guarded([&] {
    RTE_REQUIRE(h && model && bytes, RTE_EINVAL, "rte_precond_workspace_bytes: null argument");
    *bytes = precond_bytes(*h->op, *model->m);
  });
}

rte_status rte_precond_apply(const rte_operator* h, const mgnet_model* model, int precond, const double* v,
                             float* z, void* ws, size_t ws_bytes, void* stream) {
  return guarded([&] {
    RTE_REQUIRE(h && v && z, RTE_EINVAL, "rte_precond_apply: null argument");
    const Operator& o = *h->op;
    RTE_REQUIRE(o.scheme == RTE_SCHEME_UPWIND, RTE_EINVAL, "the preconditioners act on the upwind scheme");
    if (precond == RTE_PC_BLOCK_JACOBI) {
      RTE_REQUIRE(o.ndir <= RTE_BJ_MAX_DIRS, RTE_EINVAL, "Block-Jacobi supports up to 112 directions");
      launch_block_jacobi(Target::single(o), v, nullptr, z, S(stream));
      return;
    }
    RTE_REQUIRE(model && ws, RTE_EINVAL, "rte_precond_apply: null argument");
    RTE_REQUIRE(precond == RTE_PC_MGNET_BF16 || precond == RTE_PC_MGNET_FP32, RTE_EINVAL,
                "rte_precond_apply: unknown preconditioner");
    Model& m = *model->m;
    RTE_REQUIRE(o.model == &m, RTE_EINVAL, "operator was not built with this model");
    RTE_REQUIRE(ws_bytes >= precond_bytes(o, m), RTE_ENOMEM, "rte_precond_apply: workspace too small");
    RTE_REQUIRE((reinterpret_cast<uintptr_t>(ws) & 255) == 0, RTE_EINVAL, "workspace must be 256-byte aligned");
    m.ensure_on_device();
    precond_apply(Target::single(o), m, precond == RTE_PC_MGNET_FP32 ? MFMA_F32 : MFMA_BF16, v, z, static_cast<char*>(ws),
                  S(stream));
  });
}

static_assert(MGN_EPI_STORE == CONV_STORE && MGN_EPI_ACCUM == CONV_ACCUM && MGN_EPI_STORE_T == CONV_STORE_T &&
                  MGN_EPI_RESID_R == CONV_RESID_R && MGN_EPI_RESID_T == CONV_RESID_T,
              "the ABI's epilogue codes are the launcher's conv modes");
static_assert(sizeof(SlotDesc) <= 128, "mgnet_conv_apply documents 128 bytes per slot");

rte_status mgnet_conv_apply(const mgnet_model* model, int precond, int which, int level, int index,
                            int epilogue, const int* in_dim, int nslots, size_t slot_stride, const float* in,
                            float* out, float* out2, const float* f, const float* a, const float* ainv,
                            void* table, void* stream) {
  return guarded([&] {
    RTE_REQUIRE(model && in_dim && in && out, RTE_EINVAL, "mgnet_conv_apply: null argument");
    RTE_REQUIRE(precond == RTE_PC_MGNET_BF16 || precond == RTE_PC_MGNET_FP32, RTE_EINVAL,
                "mgnet_conv_apply: precond must be an MgNet precision");
    RTE_REQUIRE(epilogue >= MGN_EPI_STORE && epilogue <= MGN_EPI_RESID_T, RTE_EINVAL,
                "mgnet_conv_apply: unknown epilogue");
    RTE_REQUIRE(nslots >= 1 && (nslots == 1 || table), RTE_EINVAL, "mgnet_conv_apply: bad slot count or table");
    Model& m = *model->m;
    const int L = m.levels;
    RTE_REQUIRE(level >= 0 && level < L, RTE_EINVAL, "mgnet_conv_apply: level out of range");
    const ConvW* w = nullptr;
    auto pick = [&](const std::vector<ConvW>& v, int i) {
      RTE_REQUIRE(i >= 0 && i < int(v.size()), RTE_EINVAL, "mgnet_conv_apply: index out of range");
      return &v[size_t(i)];
    };
    const bool coarse = level == L - 1;
    switch (which) {
      case MGN_W_A: w = &m.A[size_t(level)]; break;
      case MGN_W_BPRE: RTE_REQUIRE(!coarse, RTE_EINVAL, "no B_pre on the coarsest level"); w = pick(m.Bpre[size_t(level)], index); break;
      case MGN_W_BPOST: RTE_REQUIRE(!coarse, RTE_EINVAL, "no B_post on the coarsest level"); w = pick(m.Bpost[size_t(level)], index); break;
      case MGN_W_BCOARSE: RTE_REQUIRE(coarse, RTE_EINVAL, "B_coarse lives on the coarsest level"); w = pick(m.Bc, index); break;
      case MGN_W_R: RTE_REQUIRE(!coarse, RTE_EINVAL, "no restriction from the coarsest level"); w = &m.R[size_t(level)]; break;
      case MGN_W_PR: RTE_REQUIRE(!coarse, RTE_EINVAL, "no prolongation onto the coarsest level"); w = &m.Pr[size_t(level)]; break;
      default: fail(RTE_EINVAL, "mgnet_conv_apply: unknown weights");
    }
    int d[3];
    for (int ax = 0; ax < 3; ++ax) {
      d[ax] = in_dim[ax];
      RTE_REQUIRE(d[ax] >= 1 && (ax < m.dim || d[ax] == 1), RTE_EINVAL, "mgnet_conv_apply: bad grid");
      if (ax < m.dim && which == MGN_W_R) RTE_REQUIRE(d[ax] % 2 == 0, RTE_EINVAL, "restriction needs even extents");
    }
    ConvLaunch c{};
    if (which == MGN_W_PR) convT4_setup(c, m.dim, d);
    else conv3_setup(c, m.dim, d, which == MGN_W_R ? 2 : 1);
    const bool needs_fa = epilogue == MGN_EPI_RESID_R || epilogue == MGN_EPI_RESID_T;
    const bool needs_i = epilogue == MGN_EPI_RESID_T || epilogue == MGN_EPI_STORE_T;
    RTE_REQUIRE(!needs_fa || (f && a), RTE_EINVAL, "mgnet_conv_apply: the residual epilogues need f and a");
    RTE_REQUIRE(!needs_i || ainv, RTE_EINVAL, "mgnet_conv_apply: this epilogue needs ainv");
    RTE_REQUIRE(epilogue != MGN_EPI_STORE_T || out2, RTE_EINVAL, "mgnet_conv_apply: STORE_T needs out2");
    m.ensure_on_device();
    hipStream_t s = S(stream);
    std::vector<SlotDesc> tab;
    if (table) {
      tab.assign(size_t(nslots), SlotDesc{});
      for (int z = 0; z < nslots; ++z) {
        tab[size_t(z)].ws = uint64_t(z) * slot_stride;
        tab[size_t(z)].op = uint64_t(z) * slot_stride;
        tab[size_t(z)].live = 1;
        tab[size_t(z)].occupied = 1;
      }
      RTE_HIP(hipMemcpyAsync(table, tab.data(), tab.size() * sizeof(SlotDesc), hipMemcpyHostToDevice, s));
      c.sl.tab = static_cast<SlotDesc*>(table);
      c.sl.count = nslots;
      c.sl.gate = GATE_LIVE;
    }
    c.in = in; c.cin = w->cin; c.w = w; c.out = out; c.cout = w->cout; c.mode = epilogue;
    c.f = f; c.a = a; c.ainv = ainv; c.out2 = out2;
    launch_conv(c, precond == RTE_PC_MGNET_FP32 ? MFMA_F32 : MFMA_BF16, s);
    RTE_HIP(hipStreamSynchronize(s));
  });
}

rte_status rte_workspace_bytes(const rte_operator* h, const mgnet_model* model, const rte_solve_opts* opts,
                               size_t* bytes) {
  return guarded([&] {
    RTE_REQUIRE(h && opts && bytes, RTE_EINVAL, "rte_workspace_bytes: null argument");
    const Model* m = model ? model->m.get() : nullptr;
    validate_opts(*h->op, m, opts);
    const bool mg = opts->precond == RTE_PC_MGNET_BF16 || opts->precond == RTE_PC_MGNET_FP32;
    *bytes = batch_table_bytes(1) + solve_layout(*h->op, m, opts->restart, mg).total;
  });
}

rte_status rte_solve(const rte_operator* h, const mgnet_model* model, const rte_solve_opts* opts, void* ws,
                     size_t ws_bytes, double* psi, rte_solve_stats* stats, void* stream) {
  rte_status solve_status = RTE_OK;
  rte_status st = guarded([&] {
    RTE_REQUIRE(h != nullptr && opts != nullptr, RTE_EINVAL, "rte_solve: null argument");
    const Operator& op = *h->op;
    const Model* m = model ? model->m.get() : nullptr;
    validate_opts(op, m, opts);
    RTE_REQUIRE(ws != nullptr && psi != nullptr, RTE_EINVAL, "null workspace or output");
    const size_t tb = batch_table_bytes(1);
    const bool mg = opts->precond == RTE_PC_MGNET_BF16 || opts->precond == RTE_PC_MGNET_FP32;
    const size_t need = tb + solve_layout(op, m, opts->restart, mg).total;
    RTE_REQUIRE(ws_bytes >= need, RTE_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    RTE_REQUIRE((reinterpret_cast<uintptr_t>(ws) & 255) == 0, RTE_EINVAL, "workspace must be 256-byte aligned");
    char* w = static_cast<char*>(ws);
    Batch b(op, m, opts->restart, opts->precond, 1, w, S(stream));
    b.add(nullptr, op, *opts, w + tb, psi, std::chrono::duration<double, std::milli>(
                                               std::chrono::steady_clock::now().time_since_epoch()).count());
    std::vector<Batch::Finished> done;
    while (!b.idle()) {
      b.wait();
      b.advance();
      b.collect(done);
    }
    RTE_REQUIRE(done.size() == 1, RTE_EDEVICE, "solve did not report a result");
    if (stats) *stats = done[0].stats;
    solve_status = done[0].status;
  });
  if (st != RTE_OK) return st;
  if (solve_status == RTE_ENOCONV)
    set_last_error("solve stopped before reaching rtol");
  else if (solve_status == RTE_EBREAKDOWN)
    set_last_error("non-finite values in the Krylov process");
  else if (solve_status == RTE_EINVAL)
    set_last_error("right-hand side is not finite");
  return solve_status;
}

rte_status rte_prof_enable(int c, int every) {
  return guarded([&] {
    RTE_REQUIRE(c >= 0 && c < RTE_K_COUNT, RTE_EINVAL, "unknown kernel class");
    RTE_REQUIRE(every >= 0, RTE_EINVAL, "sampling stride must be >= 0");
    Prof& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    P.every[c] = every;
    P.seen[c] = 0;
    // the events are created here, so that no timed launch creates one
    if (every > 0)
      while (P.pool.size() < kProfEventReserve) {
        hipEvent_t e;
        RTE_HIP(hipEventCreate(&e));
        P.pool.push_back(e);
      }
  });
}

rte_status rte_prof_query(int c, double* total_ms, int64_t* launches, double* work, double* bytes) {
  return guarded([&] {
    RTE_REQUIRE(c >= 0 && c < RTE_K_COUNT, RTE_EINVAL, "unknown kernel class");
    Prof& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    P.drain(c);
    if (total_ms) *total_ms = P.ms[c];
    if (launches) *launches = P.count[c];
    if (work) *work = P.work[c];
    if (bytes) *bytes = P.bytes[c];
  });
}

rte_status rte_prof_query_key(int c, int key, double* total_ms, int64_t* launches, double* work, double* bytes) {
  return guarded([&] {
    RTE_REQUIRE(c >= 0 && c < RTE_K_COUNT, RTE_EINVAL, "unknown kernel class");
    RTE_REQUIRE(key >= 0 && key < RTE_PROF_KEYS, RTE_EINVAL, "key out of range");
    Prof& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    P.drain(c);
    if (total_ms) *total_ms = P.kms[c][key];
    if (launches) *launches = P.kcount[c][key];
    if (work) *work = P.kwork[c][key];
    if (bytes) *bytes = P.kbytes[c][key];
  });
}

rte_status rte_prof_reset(void) {
  return guarded([&] {
    Prof& P = prof();
    std::lock_guard<std::mutex> lk(P.mu);
    for (int c = 0; c < RTE_K_COUNT; ++c) {
      P.drain(c);
      P.ms[c] = 0;
      P.work[c] = 0;
      P.bytes[c] = 0;
      P.count[c] = 0;
      for (int k = 0; k < RTE_PROF_KEYS; ++k) {
        P.kms[c][k] = 0;
        P.kwork[c][k] = 0;
        P.kbytes[c][k] = 0;
        P.kcount[c][k] = 0;
      }
    }
  });
}

}  // extern "C"

// Operator build on the host in FP64: validation, scattering matrix,
// diffusive scaling, right-hand side; upload; CoeffNet on the device.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace rte {

int64_t Operator::level_cells(int l) const {
  int64_t c = 1;
  for (int a = 0; a < dim; ++a) c *= level_dim(l, a);
  return c;
}

int Operator::level_dim(int l, int axis) const {
  int n = axis == 0 ? nx : axis == 1 ? ny : nz;
  if (axis >= dim) return 1;
  return n >> l;
}

std::vector<int64_t> Operator::shape_key() const {
  return {dim, nx, ny, nz, ndir, levels, c0, scheme};
}

std::unique_ptr<Operator> Operator::geometry() const {
  std::unique_ptr<Operator> o(new Operator());
  o->dim = dim;
  o->nx = nx;
  o->ny = ny;
  o->nz = nz;
  o->ndir = ndir;
  o->kernel = kernel;
  o->cells = cells;
  o->n = n;
  o->h = h;
  o->g = g;
  o->device = device;
  o->model = model;
  o->levels = levels;
  o->c0 = c0;
  o->scheme = scheme;
  o->nbasis = nbasis;
  return o;
}

OpArrays Operator::relative() const {
  auto rel = [&](auto* p) { return p ? at(p, uint64_t(0) - reinterpret_cast<uint64_t>(block)) : p; };
  OpArrays r;
  r.b64 = rel(a.b64);
  r.sT32 = rel(a.sT32);
  r.sA32 = rel(a.sA32);
  r.sT64 = rel(a.sT64);
  r.sA64 = rel(a.sA64);
  r.S32 = rel(a.S32);
  r.S64 = rel(a.S64);
  r.dc32 = rel(a.dc32);
  r.dc64 = rel(a.dc64);
  r.dsgn = rel(a.dsgn);
  r.Sdiag32 = rel(a.Sdiag32);
  r.Sp32 = rel(a.Sp32);
  for (int l = 0; l < MAX_LEVELS; ++l) {
    r.fa[l] = rel(a.fa[l]);
    r.fainv[l] = rel(a.fainv[l]);
  }
  r.tf_bid = rel(a.tf_bid);
  r.tf_chis = rel(a.tf_chis);
  r.tf_tab = rel(a.tf_tab);
  return r;
}

namespace {

// Kernel values P_mn = kappa(u_m . u_n), eq. (hg) ("sphere") or its circle
// analogue ("flatland").
std::vector<double> hg_values(const std::vector<double>& dirs, int N, double g, int kind) {
  std::vector<double> P(size_t(N) * N);
  for (int m = 0; m < N; ++m)
    for (int n = 0; n < N; ++n) {
      double mu = dirs[3 * m] * dirs[3 * n] + dirs[3 * m + 1] * dirs[3 * n + 1] +
                  dirs[3 * m + 2] * dirs[3 * n + 2];
      mu = std::min(1.0, std::max(-1.0, mu));
      double base = 1.0 + g * g - 2.0 * g * mu;
      P[size_t(m) * N + n] = kind == RTE_HG_SPHERE ? (1.0 - g * g) / (base * std::sqrt(base))
                                                    : (1.0 - g * g) / base;
    }
  return P;
}

// Scattering matrix S = D P D W with D = diag(d) chosen so that every
// w-weighted row of D P D sums to one; D P D is symmetric, so its
// w-weighted columns do too and scattering conserves particles.  Fixed
// point of d <- sqrt(d / (P W d)).
std::vector<double> scattering_matrix(const std::vector<double>& P, const std::vector<double>& w,
                                      int N) {
  std::vector<double> d(N, 1.0), nd(N), t(N);
  for (int it = 0; it < 200000; ++it) {
    double dmax = 0, change = 0;
    for (int m = 0; m < N; ++m) {
      double s = 0;
      for (int n = 0; n < N; ++n) s += P[size_t(m) * N + n] * w[n] * d[n];
      nd[m] = std::sqrt(d[m] / s);
      dmax = std::max(dmax, nd[m]);
      change = std::max(change, std::fabs(nd[m] - d[m]));
    }
    d.swap(nd);
    if (change <= 1e-15 * dmax) break;
  }
  std::vector<double> S(size_t(N) * N);
  for (int m = 0; m < N; ++m) {
    double row = 0;
    for (int n = 0; n < N; ++n) {
      S[size_t(m) * N + n] = d[m] * P[size_t(m) * N + n] * d[n] * w[n];
      row += S[size_t(m) * N + n];
    }
    RTE_REQUIRE(std::fabs(row - 1.0) < 1e-12, RTE_EINVAL,
                "scattering normalisation did not converge (row sum off by " +
                    std::to_string(row - 1.0) + ")");
  }
  return S;
}

bool finite_all(const double* p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

void build_coeffnet(Operator& op, const Model& m, const std::vector<double>& eps, hipStream_t s) {
  const int64_t cells = op.cells;
  std::vector<float> X(size_t(cells) * 3);
  std::vector<double> sT(cells), sA(cells);
  RTE_HIP(hipMemcpy(sT.data(), op.a.sT64, cells * 8, hipMemcpyDeviceToHost));
  RTE_HIP(hipMemcpy(sA.data(), op.a.sA64, cells * 8, hipMemcpyDeviceToHost));
  for (int64_t c = 0; c < cells; ++c) {
    X[3 * c + 0] = float(std::log(sT[c]));
    X[3 * c + 1] = float(sA[c] / sT[c]);
    X[3 * c + 2] = float(std::log(eps[c]));
  }
  DevArena tmp;
  const float* in = tmp.upload(X);
  int cin = 3;
  int in_dim[3] = {op.nx, op.ny, op.nz};
  for (int l = 0; l < m.levels; ++l) {
    int c = m.coef_ch << l;
    int C = m.c0 << l;
    int stride = l == 0 ? 1 : 2;
    int out_dim[3] = {op.level_dim(l, 0), op.level_dim(l, 1), op.level_dim(l, 2)};
    int64_t P = op.level_cells(l);
    float* F = tmp.alloc<float>(size_t(P) * c);
    launch_coef_conv(in, cin, in_dim, m.d_CW[l], m.d_CB[l], F, c, out_dim, op.dim, stride, s);
    launch_head(F, c, m.d_HAW[l], m.d_HAB[l], op.a.fa[l], C, P, s);
    launch_head(F, c, m.d_HIW[l], m.d_HIB[l], op.a.fainv[l], C, P, s);
    in = F;
    cin = c;
    for (int a2 = 0; a2 < 3; ++a2) in_dim[a2] = out_dim[a2];
  }
  RTE_HIP(hipStreamSynchronize(s));
}

}  // namespace

Operator* build_operator(const rte_geometry* g, const rte_medium* md, const Model* model,
                         hipStream_t stream) {
  RTE_REQUIRE(g && md, RTE_EINVAL, "rte_build_operator: null geometry or medium");
  RTE_REQUIRE(g->dim == 2 || g->dim == 3, RTE_EINVAL, "dim must be 2 or 3");
  const int dim = g->dim;
  const int nx = g->n[0], ny = g->n[1], nz = dim == 3 ? g->n[2] : 1;
  RTE_REQUIRE(nx >= 1 && nx <= 4096, RTE_EINVAL, "cells per axis must be in [1, 4096]");
  RTE_REQUIRE(ny == nx && (dim == 2 || nz == nx), RTE_EINVAL,
              "cubic cells on the unit square/cube need equal cell counts per axis");
  RTE_REQUIRE(dim == 3 || g->n[2] <= 1, RTE_EINVAL, "n[2] must be 1 (or 0) in 2D");
  const int N = g->ndir;
  RTE_REQUIRE(N >= 1 && N <= 256, RTE_EINVAL, "ndir must be in [1, 256]");
  RTE_REQUIRE(g->dirs && g->weights, RTE_EINVAL, "null directions or weights");
  RTE_REQUIRE(std::isfinite(g->g) && std::fabs(g->g) < 1.0, RTE_EINVAL, "|g| must be < 1");
  RTE_REQUIRE(g->kernel >= 0 && g->kernel <= 2, RTE_EINVAL, "unknown kernel kind");
  std::vector<double> dirs(g->dirs, g->dirs + 3 * N), w(g->weights, g->weights + N);
  RTE_REQUIRE(finite_all(dirs.data(), 3 * N) && finite_all(w.data(), N), RTE_EINVAL,
              "non-finite direction or weight");
  double wsum = 0;
  bool flat = true;
  for (int m = 0; m < N; ++m) {
    double nrm = std::sqrt(dirs[3 * m] * dirs[3 * m] + dirs[3 * m + 1] * dirs[3 * m + 1] +
                           dirs[3 * m + 2] * dirs[3 * m + 2]);
    RTE_REQUIRE(std::fabs(nrm - 1.0) <= 1e-12, RTE_EINVAL, "direction " + std::to_string(m) + " is not a unit vector");
    RTE_REQUIRE(w[m] > 0, RTE_EINVAL, "weights must be positive");
    wsum += w[m];
    if (dirs[3 * m + 2] != 0.0) flat = false;
  }
  RTE_REQUIRE(std::fabs(wsum - 1.0) <= 1e-12, RTE_EINVAL, "weights must sum to 1");
  const int kind = g->kernel == RTE_HG_AUTO ? (flat ? RTE_HG_FLATLAND : RTE_HG_SPHERE) : g->kernel;

  const int64_t cells = int64_t(nx) * ny * nz;
  RTE_REQUIRE(md->sigma_t && md->sigma_a && md->q, RTE_EINVAL, "null medium array");
  RTE_REQUIRE(int64_t(N) * cells <= (int64_t(1) << 31) - 1, RTE_EINVAL, "problem too large (n >= 2^31)");
  std::vector<double> eps(cells);
  for (int64_t c = 0; c < cells; ++c) eps[c] = md->eps ? md->eps[c] : md->eps_scalar;
  for (int64_t c = 0; c < cells; ++c) {
    double st = md->sigma_t[c], sa = md->sigma_a[c], q = md->q[c], e = eps[c];
    RTE_REQUIRE(std::isfinite(st) && std::isfinite(sa) && std::isfinite(q) && std::isfinite(e),
                RTE_EINVAL, "non-finite medium value at cell " + std::to_string(c));
    RTE_REQUIRE(st > 0, RTE_EINVAL, "sigma_t must be > 0");
    RTE_REQUIRE(sa >= 0 && q >= 0, RTE_EINVAL, "sigma_a and q must be >= 0");
    RTE_REQUIRE(e > 0 && e <= 1, RTE_EINVAL, "eps must lie in (0, 1]");
    RTE_REQUIRE(st / e - e * sa >= 0, RTE_EINVAL,
                "sigma_t/eps - eps*sigma_a < 0 at cell " + std::to_string(c) + " (negative scattering)");
  }
  RTE_REQUIRE(g->scheme == RTE_SCHEME_UPWIND || g->scheme == RTE_SCHEME_TFPS, RTE_EINVAL, "unknown scheme");
  const bool tfps = g->scheme == RTE_SCHEME_TFPS;
  if (tfps) {
    RTE_REQUIRE(dim == 2, RTE_EINVAL, "the TFPS operator is two-dimensional");
    RTE_REQUIRE(model == nullptr, RTE_EINVAL, "MgNet preconditions the upwind scheme; build TFPS without a model");
    RTE_REQUIRE(int64_t(2) * N * cells <= (int64_t(1) << 31) - 1, RTE_EINVAL, "problem too large (n >= 2^31)");
  }
  if (model) {
    RTE_REQUIRE(model->dim == dim && model->ndir == N, RTE_EINVAL, "model does not match the geometry");
    int div = 1 << (model->levels - 1);
    RTE_REQUIRE(nx % div == 0, RTE_EINVAL, "grid extent not divisible by 2^(levels-1) of the model");
    RTE_REQUIRE(model->levels <= MAX_LEVELS, RTE_EINVAL, "too many MgNet levels");
  }

  Operator* op = new Operator();
  try {
    op->dim = dim; op->nx = nx; op->ny = ny; op->nz = nz; op->ndir = N; op->kernel = kind;
    op->cells = cells; op->n = int64_t(tfps ? 2 : 1) * N * cells; op->h = 1.0 / nx; op->g = g->g;
    op->scheme = g->scheme;
    RTE_HIP(hipGetDevice(&op->device));
    op->S = scattering_matrix(hg_values(dirs, N, g->g, kind), w, N);

    std::vector<double> sT(cells), sA(cells);
    for (int64_t c = 0; c < cells; ++c) {
      sT[c] = md->sigma_t[c] / eps[c];
      sA[c] = eps[c] * md->sigma_a[c];
    }
    // per direction streaming coefficients |u_a|/h and upwind signs
    std::vector<double> dc(size_t(N) * 4, 0.0);
    std::vector<int> sg(size_t(N) * 4, 0);
    for (int m = 0; m < N; ++m) {
      double sum = 0;
      for (int a = 0; a < dim; ++a) {
        double u = dirs[3 * m + a];
        dc[4 * m + a] = std::fabs(u) / op->h;
        sg[4 * m + a] = u > 0 ? 1 : (u < 0 ? -1 : 0);
        sum += dc[4 * m + a];
      }
      dc[4 * m + 3] = sum;
    }
    // right-hand side: eps q plus the inflow flux through boundary faces
    size_t fstride = md->inflow_face_stride;
    if (fstride == 0) fstride = size_t(std::max({int64_t(ny) * nz, int64_t(nx) * nz, dim == 3 ? int64_t(nx) * ny : 0}));
    if (md->inflow)
      RTE_REQUIRE(finite_all(md->inflow, int64_t(2 * dim) * N * int64_t(fstride)), RTE_EINVAL,
                  "non-finite inflow value");
    TfpsHost TF;
    std::vector<double> b;
    if (tfps) {
      std::vector<double> qh(cells);
      for (int64_t c = 0; c < cells; ++c) qh[c] = eps[c] * md->q[c];
      TF = tfps_build_host(*op, dirs, w, sT, sA, qh, md->inflow, fstride);
      op->nbasis = TF.nbasis;
      b = TF.b;
    } else {
      b.assign(size_t(op->n), 0.0);
      for (int m = 0; m < N; ++m)
        for (int64_t c = 0; c < cells; ++c) b[size_t(m) * cells + c] = eps[c] * md->q[c];
    }
    if (md->inflow && !tfps) {
      for (int m = 0; m < N; ++m)
        for (int a = 0; a < dim; ++a) {
          int sgn = sg[4 * m + a];
          if (sgn == 0) continue;
          int face = 2 * a + (sgn > 0 ? 0 : 1);
          const double* F = md->inflow + (size_t(face) * N + m) * fstride;
          double coef = dc[4 * m + a];
          for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j)
              for (int i = 0; i < nx; ++i) {
                int idx[3] = {i, j, k};
                int ext[3] = {nx, ny, nz};
                if (idx[a] != (sgn > 0 ? 0 : ext[a] - 1)) continue;
                size_t fi = a == 0 ? size_t(k) * ny + j : a == 1 ? size_t(k) * nx + i : size_t(j) * nx + i;
                b[size_t(m) * cells + (int64_t(k) * ny + j) * nx + i] += coef * F[fi];
              }
        }
    }
    std::vector<float> sT32(cells), sA32(cells), S32(size_t(N) * N), dc32(dc.size()), Sd(N);
    for (int64_t c = 0; c < cells; ++c) {
      sT32[c] = float(sT[c]);
      sA32[c] = float(sA[c]);
    }
    for (size_t i = 0; i < S32.size(); ++i) S32[i] = float(op->S[i]);
    for (size_t i = 0; i < dc.size(); ++i) dc32[i] = float(dc[i]);
    for (int m = 0; m < N; ++m) Sd[m] = float(op->S[size_t(m) * N + m]);
    // one device block, laid out by shape only
    if (model) {
      op->levels = model->levels;
      op->c0 = model->c0;
    }
    size_t off = 256;
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off += (bytes + 255) & ~size_t(255);
      return o;
    };
    const size_t o_b = take(size_t(op->n) * 8), o_sT64 = take(cells * 8), o_sA64 = take(cells * 8);
    const size_t o_sT32 = take(cells * 4), o_sA32 = take(cells * 4);
    const size_t o_S64 = take(size_t(N) * N * 8), o_S32 = take(size_t(N) * N * 4);
    const size_t o_dc64 = take(dc.size() * 8), o_dc32 = take(dc.size() * 4), o_sg = take(sg.size() * 4);
    const size_t o_sd = take(size_t(N) * 4);
    // S packed by direction slot for the one-slot-per-wave apply
    const int dp = slot_budget(N);
    std::vector<float> Sp(size_t(4) * N * (dp > 0 ? dp : 0), 0.f);
    for (int sl = 0; sl < 4 && dp > 0; ++sl)
      for (int n = 0; n < N; ++n)
        for (int q = 0; q < dp; ++q) {
          const int m = sl + 4 * q;
          if (m < N) Sp[(size_t(sl) * N + n) * dp + q] = float(op->S[size_t(m) * N + n]);
        }
    const size_t o_sp = take(Sp.size() * 4);
    size_t o_fa[MAX_LEVELS] = {}, o_fi[MAX_LEVELS] = {};
    for (int l = 0; l < op->levels; ++l) {
      const size_t bytes = size_t(op->level_cells(l)) * (op->c0 << l) * 4;
      o_fa[l] = take(bytes);
      o_fi[l] = take(bytes);
    }
    size_t o_bid = 0, o_chis = 0, o_tab = 0;
    if (tfps) {
      o_bid = take(size_t(cells) * 4);
      o_chis = take(size_t(cells) * 8);
      o_tab = take(16);
    }
    op->block_bytes = off;
    op->block = op->mem.alloc<char>(off);
    char* B = op->block;
    auto put = [&](size_t o, const void* src, size_t bytes) {
      RTE_HIP(hipMemcpy(B + o, src, bytes, hipMemcpyHostToDevice));
      return B + o;
    };
    op->a.b64 = reinterpret_cast<double*>(put(o_b, b.data(), b.size() * 8));
    op->a.sT64 = reinterpret_cast<double*>(put(o_sT64, sT.data(), cells * 8));
    op->a.sA64 = reinterpret_cast<double*>(put(o_sA64, sA.data(), cells * 8));
    op->a.sT32 = reinterpret_cast<float*>(put(o_sT32, sT32.data(), cells * 4));
    op->a.sA32 = reinterpret_cast<float*>(put(o_sA32, sA32.data(), cells * 4));
    op->a.S64 = reinterpret_cast<double*>(put(o_S64, op->S.data(), op->S.size() * 8));
    op->a.S32 = reinterpret_cast<float*>(put(o_S32, S32.data(), S32.size() * 4));
    op->a.dc64 = reinterpret_cast<double*>(put(o_dc64, dc.data(), dc.size() * 8));
    op->a.dc32 = reinterpret_cast<float*>(put(o_dc32, dc32.data(), dc32.size() * 4));
    op->a.dsgn = reinterpret_cast<int*>(put(o_sg, sg.data(), sg.size() * 4));
    op->a.Sdiag32 = reinterpret_cast<float*>(put(o_sd, Sd.data(), Sd.size() * 4));
    if (!Sp.empty()) op->a.Sp32 = reinterpret_cast<float*>(put(o_sp, Sp.data(), Sp.size() * 4));
    for (int l = 0; l < op->levels; ++l) {
      op->a.fa[l] = reinterpret_cast<float*>(B + o_fa[l]);
      op->a.fainv[l] = reinterpret_cast<float*>(B + o_fi[l]);
    }
    if (tfps) {
      // the basis tables live outside the block (their size depends on the medium);
      // the block holds their addresses
      const double* dL = op->mem.upload(TF.Lt);
      const double* dxi = op->mem.upload(TF.xi);
      const uint64_t tabs[2] = {reinterpret_cast<uint64_t>(dL), reinterpret_cast<uint64_t>(dxi)};
      op->a.tf_bid = reinterpret_cast<int*>(put(o_bid, TF.bid.data(), TF.bid.size() * 4));
      op->a.tf_chis = reinterpret_cast<double*>(put(o_chis, TF.chis.data(), TF.chis.size() * 8));
      op->a.tf_tab = reinterpret_cast<uint64_t*>(put(o_tab, tabs, sizeof(tabs)));
      op->tfps_host = std::make_shared<const TfpsHost>(std::move(TF));
    }
    if (model) {
      const_cast<Model*>(model)->ensure_on_device();
      build_coeffnet(*op, *model, eps, stream);
      op->model = model;
    }
  } catch (...) {
    delete op;
    throw;
  }
  return op;
}

}  // namespace rte

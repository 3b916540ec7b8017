// Host FP64 build of the tailored finite point scheme (Sec. 2.2): the
// per-cell eigen-bases of eq. (discretization_2D_eigenfunc_constraint), the
// particular solutions and the right-hand side of eq. (2DTFPS_linear_sys).
//
// In a cell with ratio a = sS/sT the x-type modes solve
//   (a S - I) l = xi Cx l,      S = K W (K symmetric, W = diag(w) > 0),
// Cx = diag(u_x).  With v = W^{1/2} l the problem becomes the symmetric
// pencil (a W^{1/2} K W^{1/2} - I) v = xi Cx v, whose left side is negative
// definite (the eigenvalues of S lie in [-1, 1] and a < 1 since sA > 0).  With
// M = I - a W^{1/2} K W^{1/2} = Lc Lc^T (Cholesky),
//   H = Lc^{-1} Cx Lc^{-T} is symmetric, H y = mu y, xi = -1/mu,
//   v = Lc^{-T} y,  l = W^{-1/2} v,
// and H is diagonalised by cyclic Jacobi rotations.  The y-type modes are the
// same with Cy.  Cells with equal a share one basis.
#include <algorithm>
#include <cmath>
#include <thread>
#include <unordered_map>

#include "common.h"

namespace rte {
namespace {

// Eigenvalues (returned) and eigenvectors (columns of V, row-major n x n) of
// the symmetric matrix A (row-major, destroyed), by cyclic Jacobi sweeps.
std::vector<double> jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& V) {
  V.assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) V[size_t(i) * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[size_t(i) * n + j]; };
  double scale = 0;
  for (double x : A) scale = std::max(scale, std::fabs(x));
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off = std::max(off, std::fabs(a(p, q)));
    if (off <= 1e-17 * scale) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (apq == 0.0) continue;
        // rotation zeroing a(p, q): t = tan(angle), the smaller root of t^2 + 2 th t - 1 = 0
        const double th = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - s * akq;
          a(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - s * aqk;
          a(q, k) = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[size_t(k) * n + p], vkq = V[size_t(k) * n + q];
          V[size_t(k) * n + p] = c * vkp - s * vkq;
          V[size_t(k) * n + q] = s * vkp + c * vkq;
        }
      }
  }
  std::vector<double> ev(n);
  for (int i = 0; i < n; ++i) ev[i] = a(i, i);
  return ev;
}

// Modes along one axis (u = that component of every direction): xi ascending
// and the matching eigenvectors l (columns of Lm, row-major N x N), each of
// max-norm 1 with its first entry within 1e-8 of the largest magnitude positive.
void axis_modes(int N, const std::vector<double>& S, const std::vector<double>& w, double a,
                const std::vector<double>& u, std::vector<double>& xi, std::vector<double>& Lm) {
  // M = I - a W^{1/2} K W^{1/2}; with K_mn = S_mn / w_n: entry S_mn sqrt(w_m / w_n)
  std::vector<double> M(size_t(N) * N);
  for (int m = 0; m < N; ++m)
    for (int n = 0; n < N; ++n)
      M[size_t(m) * N + n] = (m == n ? 1.0 : 0.0) - a * S[size_t(m) * N + n] * std::sqrt(w[m] / w[n]);
  // symmetrise against rounding, then Cholesky M = Lc Lc^T (Lc lower, in place)
  for (int m = 0; m < N; ++m)
    for (int n = m + 1; n < N; ++n) {
      const double v = 0.5 * (M[size_t(m) * N + n] + M[size_t(n) * N + m]);
      M[size_t(m) * N + n] = M[size_t(n) * N + m] = v;
    }
  std::vector<double> Lc(size_t(N) * N, 0.0);
  for (int j = 0; j < N; ++j) {
    double d = M[size_t(j) * N + j];
    for (int k = 0; k < j; ++k) d -= Lc[size_t(j) * N + k] * Lc[size_t(j) * N + k];
    RTE_REQUIRE(d > 0, RTE_EINVAL, "TFPS: I - a S is not positive definite (needs sigma_a > 0)");
    const double ljj = std::sqrt(d);
    Lc[size_t(j) * N + j] = ljj;
    for (int i = j + 1; i < N; ++i) {
      double v = M[size_t(i) * N + j];
      for (int k = 0; k < j; ++k) v -= Lc[size_t(i) * N + k] * Lc[size_t(j) * N + k];
      Lc[size_t(i) * N + j] = v / ljj;
    }
  }
  // X = Lc^{-1} diag(u) (forward substitution, column by column), H = X Lc^{-T} = (Lc^{-1} X^T)^T
  std::vector<double> X(size_t(N) * N, 0.0), H(size_t(N) * N, 0.0);
  auto lsolve = [&](std::vector<double>& B) {  // B <- Lc^{-1} B (B row-major N x N)
    for (int col = 0; col < N; ++col)
      for (int i = 0; i < N; ++i) {
        double v = B[size_t(i) * N + col];
        for (int k = 0; k < i; ++k) v -= Lc[size_t(i) * N + k] * B[size_t(k) * N + col];
        B[size_t(i) * N + col] = v / Lc[size_t(i) * N + i];
      }
  };
  for (int i = 0; i < N; ++i) X[size_t(i) * N + i] = u[i];
  lsolve(X);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) H[size_t(i) * N + j] = X[size_t(j) * N + i];  // X^T
  lsolve(H);                                                                     // Lc^{-1} X^T = H^T = H
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j) {
      const double v = 0.5 * (H[size_t(i) * N + j] + H[size_t(j) * N + i]);
      H[size_t(i) * N + j] = H[size_t(j) * N + i] = v;
    }
  std::vector<double> Y;
  std::vector<double> mu = jacobi_eigen(N, H, Y);
  // v = Lc^{-T} y (back substitution), l = W^{-1/2} v
  std::vector<std::pair<double, int>> order(N);
  for (int k = 0; k < N; ++k) {
    RTE_REQUIRE(mu[k] != 0.0, RTE_EINVAL, "TFPS: zero mode (a direction with a zero component)");
    order[k] = {-1.0 / mu[k], k};
  }
  std::sort(order.begin(), order.end());
  xi.assign(N, 0.0);
  Lm.assign(size_t(N) * N, 0.0);
  std::vector<double> v(N);
  for (int c = 0; c < N; ++c) {
    const int k = order[c].second;
    xi[c] = order[c].first;
    for (int i = N - 1; i >= 0; --i) {
      double s = Y[size_t(i) * N + k];
      for (int r = i + 1; r < N; ++r) s -= Lc[size_t(r) * N + i] * v[r];
      v[i] = s / Lc[size_t(i) * N + i];
    }
    double big = 0;
    for (int i = 0; i < N; ++i) {
      v[i] /= std::sqrt(w[i]);
      big = std::max(big, std::fabs(v[i]));
    }
    int first = 0;
    while (std::fabs(v[first]) < (1.0 - 1e-8) * big) ++first;
    const double sc = (v[first] > 0 ? 1.0 : -1.0) / big;
    for (int i = 0; i < N; ++i) Lm[size_t(i) * N + c] = v[i] * sc;
  }
}

}  // namespace

TfpsHost tfps_build_host(const Operator& op, const std::vector<double>& dirs, const std::vector<double>& w,
                         const std::vector<double>& sT, const std::vector<double>& sA,
                         const std::vector<double>& qh, const double* inflow, size_t fstride) {
  const int N = op.ndir, I = op.nx;
  const int64_t cells = op.cells;
  std::vector<double> ux(N), uy(N);
  int px = 0, py = 0;
  for (int m = 0; m < N; ++m) {
    ux[m] = dirs[3 * m];
    uy[m] = dirs[3 * m + 1];
    RTE_REQUIRE(ux[m] != 0.0 && uy[m] != 0.0, RTE_EINVAL, "TFPS: every direction needs nonzero x and y components");
    px += ux[m] > 0;
    py += uy[m] > 0;
  }
  RTE_REQUIRE(2 * px == N && 2 * py == N, RTE_EINVAL, "TFPS: half of the directions must point each way along x and y");
  TfpsHost H;
  H.sT = sT;
  H.ux = ux;
  H.uy = uy;
  H.bid.assign(size_t(cells), 0);
  H.chis.assign(size_t(cells), 0.0);
  std::unordered_map<double, int> ids;
  std::vector<double> ratios;
  for (int64_t c = 0; c < cells; ++c) {
    RTE_REQUIRE(sA[c] > 0, RTE_EINVAL, "TFPS needs sigma_a > 0 in every cell");
    const double a = (sT[c] - sA[c]) / sT[c];  // sS / sT
    auto it = ids.find(a);
    if (it == ids.end()) {
      it = ids.emplace(a, int(ratios.size())).first;
      ratios.push_back(a);
    }
    H.bid[c] = it->second;
    H.chis[c] = qh[c] / sA[c];
  }
  const int nb = int(ratios.size());
  H.nbasis = nb;
  H.Lt.assign(size_t(nb) * 2 * N * N, 0.0);
  H.xi.assign(size_t(nb) * 2 * N, 0.0);
  auto one = [&](int b) {
    std::vector<double> xi, Lm;
    for (int ax = 0; ax < 2; ++ax) {
      axis_modes(N, op.S, w, ratios[b], ax == 0 ? ux : uy, xi, Lm);
      for (int c = 0; c < N; ++c) {
        const int k = ax * N + c;  // local order: x-type then y-type, each ascending (negatives first)
        H.xi[size_t(b) * 2 * N + k] = xi[c];
        for (int m = 0; m < N; ++m) H.Lt[(size_t(b) * 2 * N + k) * N + m] = Lm[size_t(m) * N + c];
      }
      int neg = 0;
      for (int c = 0; c < N; ++c) neg += xi[c] < 0;
      RTE_REQUIRE(2 * neg == N, RTE_EINVAL, "TFPS: eigenvalues do not split evenly by sign");
    }
  };
  const int nthr = std::max(1, std::min<int>(int(std::thread::hardware_concurrency()), std::min(nb, 32)));
  if (nthr <= 1 || nb < 8) {
    for (int b = 0; b < nb; ++b) one(b);
  } else {
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> err(static_cast<size_t>(nthr));
    for (int t = 0; t < nthr; ++t)
      th.emplace_back([&, t] {
        try {
          for (int b = t; b < nb; b += nthr) one(b);
        } catch (...) {
          err[size_t(t)] = std::current_exception();
        }
      });
    for (auto& x : th) x.join();
    for (auto& e : err)
      if (e) std::rethrow_exception(e);
  }
  // right-hand side, cell-major [cells][2][N]
  H.b.assign(size_t(cells) * 2 * N, 0.0);
  auto face = [&](int f, int m, int idx) -> double {
    return inflow ? inflow[(size_t(f) * N + m) * fstride + size_t(idx)] : 0.0;
  };
  for (int j = 0; j < I; ++j)
    for (int i = 0; i < I; ++i) {
      const int64_t c = int64_t(j) * I + i;
      double* bx = &H.b[size_t(c) * 2 * N];
      double* by = bx + N;
      for (int m = 0; m < N; ++m) {
        if (i >= 1) bx[m] = H.chis[c] - H.chis[c - 1];
        else if (ux[m] > 0) bx[m] = face(0, m, j) - H.chis[c];
        else bx[m] = face(1, m, j) - H.chis[int64_t(j) * I + I - 1];
        if (j >= 1) by[m] = H.chis[c] - H.chis[c - I];
        else if (uy[m] > 0) by[m] = face(2, m, i) - H.chis[c];
        else by[m] = face(3, m, i) - H.chis[int64_t(I - 1) * I + i];
      }
    }
  return H;
}

}  // namespace rte

// Host FP64 build of the adaptive tailored finite point scheme (Sec. 2.3)
// on top of a TFPS operator: selection of the slowly decaying basis
// functions (eq. (def_V_delta)), the interface bases, the compressed system
// of eq. (2DAdaptiveTFPS_linear_sys), the layer reconstruction of eq.
// (2DAdaptive_TFPS_layer1) and (2DAdaptive_TFPS_layer2), and the filtered
// loss of eq. (loss_delta).  Each of the three linear maps the device
// evaluates is assembled here as a sparse matrix plus a constant:
//   compressed residual   r = b_d - A_d alpha
//   reconstruction        coef = R alpha + r0   (all 2N coefficients per cell)
//   filtered loss         rho = c0 - M psi, loss = ||rho||_2, M = A_d D_d,
//                         c0 = b_d - A_d d0, with alpha = D_d psi + d0 the
//                         per-cell minimum-norm least-squares fit of the
//                         cell-centre values minus the particular solution.
// Face order, row order and the interface bases follow the scheme's
// definition: x faces x_0..x_I of each grid row, then y faces y_0..y_I of
// each grid column; per face the kept functions centred on it (left or lower
// cell first, local index ascending) orthonormalised by a Householder QR and
// scaled to max-norm 1 (first entry within 1e-8 of the largest magnitude
// positive), then the dropped functions' eigenvectors scaled to max-norm 1.
#include <algorithm>
#include <cmath>
#include <exception>
#include <thread>

#include "common.h"

namespace rte {
namespace {

// Thin Householder QR of the m x n (n <= m) matrix A (row-major): Q (m x n,
// row-major) and R (n x n upper, row-major).
void householder_qr(int m, int n, const std::vector<double>& A, std::vector<double>& Q, std::vector<double>& R) {
  std::vector<double> W = A;  // overwritten by R in its upper part
  std::vector<std::vector<double>> vs;
  for (int k = 0; k < n; ++k) {
    double nrm = 0;
    for (int i = k; i < m; ++i) nrm += W[size_t(i) * n + k] * W[size_t(i) * n + k];
    nrm = std::sqrt(nrm);
    std::vector<double> v(size_t(m - k), 0.0);
    const double akk = W[size_t(k) * n + k];
    const double alpha = akk >= 0 ? -nrm : nrm;
    for (int i = k; i < m; ++i) v[size_t(i - k)] = W[size_t(i) * n + k];
    v[0] -= alpha;
    double vn = 0;
    for (double x : v) vn += x * x;
    if (vn > 0) {
      for (int j = k; j < n; ++j) {
        double d = 0;
        for (int i = k; i < m; ++i) d += v[size_t(i - k)] * W[size_t(i) * n + j];
        const double f = 2.0 * d / vn;
        for (int i = k; i < m; ++i) W[size_t(i) * n + j] -= f * v[size_t(i - k)];
      }
    }
    vs.push_back(std::move(v));
  }
  R.assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) R[size_t(i) * n + j] = W[size_t(i) * n + j];
  // Q = H_0 H_1 ... H_{n-1} applied to the first n columns of the identity
  Q.assign(size_t(m) * n, 0.0);
  for (int j = 0; j < n; ++j) Q[size_t(j) * n + j] = 1.0;
  for (int k = n - 1; k >= 0; --k) {
    const std::vector<double>& v = vs[size_t(k)];
    double vn = 0;
    for (double x : v) vn += x * x;
    if (vn == 0) continue;
    for (int j = 0; j < n; ++j) {
      double d = 0;
      for (int i = k; i < m; ++i) d += v[size_t(i - k)] * Q[size_t(i) * n + j];
      const double f = 2.0 * d / vn;
      for (int i = k; i < m; ++i) Q[size_t(i) * n + j] -= f * v[size_t(i - k)];
    }
  }
}

// Inverse of the n x n matrix A (row-major) by LU with partial pivoting.
std::vector<double> lu_inverse(int n, std::vector<double> A) {
  std::vector<int> piv(static_cast<size_t>(n));
  for (int i = 0; i < n; ++i) piv[size_t(i)] = i;
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[size_t(i) * n + k]) > std::fabs(A[size_t(p) * n + k])) p = i;
    RTE_REQUIRE(A[size_t(p) * n + k] != 0.0, RTE_EINVAL, "ATFPS: singular interface basis");
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A[size_t(k) * n + j], A[size_t(p) * n + j]);
      std::swap(piv[size_t(k)], piv[size_t(p)]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = A[size_t(i) * n + k] / A[size_t(k) * n + k];
      A[size_t(i) * n + k] = f;
      for (int j = k + 1; j < n; ++j) A[size_t(i) * n + j] -= f * A[size_t(k) * n + j];
    }
  }
  std::vector<double> inv(size_t(n) * n, 0.0), col(static_cast<size_t>(n));
  for (int c = 0; c < n; ++c) {
    for (int i = 0; i < n; ++i) col[size_t(i)] = piv[size_t(i)] == c ? 1.0 : 0.0;
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < i; ++k) col[size_t(i)] -= A[size_t(i) * n + k] * col[size_t(k)];
    for (int i = n - 1; i >= 0; --i) {
      for (int k = i + 1; k < n; ++k) col[size_t(i)] -= A[size_t(i) * n + k] * col[size_t(k)];
      col[size_t(i)] /= A[size_t(i) * n + i];
    }
    for (int i = 0; i < n; ++i) inv[size_t(i) * n + c] = col[size_t(i)];
  }
  return inv;
}

// Minimum-norm least-squares inverse (n x m, row-major) of the m x n matrix M
// (row-major), from its singular value decomposition by one-sided Jacobi
// rotations on the tall orientation (M, or M^T when n > m).  Singular values
// at or below 2^-52 max(m, n) sigma_max are taken as zero, so a rank-deficient
// fit (kept functions that coincide at the centre) gets the minimum-norm
// solution instead of an overflow.
std::vector<double> pseudo_inverse(int m, int n, const std::vector<double>& M) {
  const bool tall = n <= m;
  const int r = tall ? m : n, k = tall ? n : m;  // A is r x k, k <= r
  std::vector<double> A(size_t(r) * k), V(size_t(k) * k, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      const double x = M[size_t(i) * n + j];
      if (tall)
        A[size_t(i) * k + j] = x;
      else
        A[size_t(j) * k + i] = x;
    }
  for (int j = 0; j < k; ++j) V[size_t(j) * k + j] = 1.0;
  // rotate column pairs until every pair is orthogonal to working precision
  for (int sweep = 0; sweep < 80; ++sweep) {
    bool rotated = false;
    for (int p = 0; p + 1 < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        double a = 0, b = 0, g = 0;
        for (int i = 0; i < r; ++i) {
          const double x = A[size_t(i) * k + p], y = A[size_t(i) * k + q];
          a += x * x;
          b += y * y;
          g += x * y;
        }
        if (g == 0.0 || std::fabs(g) <= 1e-15 * std::sqrt(a * b)) continue;
        rotated = true;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < r; ++i) {
          const double x = A[size_t(i) * k + p], y = A[size_t(i) * k + q];
          A[size_t(i) * k + p] = c * x - sn * y;
          A[size_t(i) * k + q] = sn * x + c * y;
        }
        for (int i = 0; i < k; ++i) {
          const double x = V[size_t(i) * k + p], y = V[size_t(i) * k + q];
          V[size_t(i) * k + p] = c * x - sn * y;
          V[size_t(i) * k + q] = sn * x + c * y;
        }
      }
    if (!rotated) break;
  }
  // columns of A are sigma_j u_j; pinv(A) = sum_j v_j (sigma_j u_j)^T / sigma_j^2
  std::vector<double> s2(static_cast<size_t>(k), 0.0);
  double smax = 0;
  for (int j = 0; j < k; ++j) {
    for (int i = 0; i < r; ++i) s2[size_t(j)] += A[size_t(i) * k + j] * A[size_t(i) * k + j];
    smax = std::max(smax, std::sqrt(s2[size_t(j)]));
  }
  const double cut = std::ldexp(1.0, -52) * std::max(m, n) * smax;
  std::vector<double> P(size_t(n) * m, 0.0);
  for (int j = 0; j < k; ++j) {
    if (!(std::sqrt(s2[size_t(j)]) > cut)) continue;
    const double inv = 1.0 / s2[size_t(j)];
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < r; ++b) {
        const double v = V[size_t(a) * k + j] * A[size_t(b) * k + j] * inv;  // pinv(A)[a][b]
        if (tall)
          P[size_t(a) * m + b] += v;  // n x m with a < n, b < m
        else
          P[size_t(b) * m + a] += v;  // pinv(M) = pinv(M^T)^T
      }
  }
  return P;
}

// fn(i) for i in [0, count) on the host's threads (contiguous ranges; each
// index writes only its own outputs); the first exception is rethrown.
template <class F>
void parallel_for(int64_t count, F fn) {
  const int nthr = int(std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(count / 64, 32),
                                                              int64_t(std::thread::hardware_concurrency()))));
  if (nthr <= 1) {
    for (int64_t i = 0; i < count; ++i) fn(i);
    return;
  }
  std::vector<std::thread> th;
  std::vector<std::exception_ptr> err(static_cast<size_t>(nthr));
  for (int t = 0; t < nthr; ++t)
    th.emplace_back([&, t] {
      try {
        const int64_t b = count * t / nthr, e = count * (t + 1) / nthr;
        for (int64_t i = b; i < e; ++i) fn(i);
      } catch (...) {
        err[size_t(t)] = std::current_exception();
      }
    });
  for (auto& x : th) x.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

void maxnorm_columns(int m, int n, std::vector<double>& V, bool fix_sign) {
  for (int k = 0; k < n; ++k) {
    double big = 0;
    for (int i = 0; i < m; ++i) big = std::max(big, std::fabs(V[size_t(i) * n + k]));
    if (big == 0) continue;
    double sc = 1.0 / big;
    if (fix_sign) {
      int first = 0;
      while (std::fabs(V[size_t(first) * n + k]) < (1.0 - 1e-8) * big) ++first;
      if (V[size_t(first) * n + k] < 0) sc = -sc;
    }
    for (int i = 0; i < m; ++i) V[size_t(i) * n + k] *= sc;
  }
}


}  // namespace

AtfpsHost atfps_build_host(const Operator& op, double delta) {
  RTE_REQUIRE(op.scheme == RTE_SCHEME_TFPS && op.tfps_host, RTE_EINVAL, "ATFPS is built on a TFPS operator");
  RTE_REQUIRE(std::isfinite(delta) && delta >= 0 && delta < 1, RTE_EINVAL, "delta must lie in [0, 1)");
  const TfpsHost& T = *op.tfps_host;
  const int N = op.ndir, I = op.nx, K = 2 * N, hN = N / 2;
  const int64_t cells = op.cells;
  const double h = op.h;
  AtfpsHost out;
  out.cells = cells;
  out.ndir = N;
  // per cell: basis table, exponential factors at the four faces and the centre
  auto Lval = [&](int64_t c, int m, int k) {  // eigenvector k of cell c, entry m
    return T.Lt[(size_t(T.bid[size_t(c)]) * K + k) * N + m];
  };
  auto xi = [&](int64_t c, int k) { return T.xi[size_t(T.bid[size_t(c)]) * K + k]; };
  auto efac = [&](int64_t c, int k, int f) {  // f: 0 left 1 right 2 bottom 3 top 4 centre
    const double a = T.sT[size_t(c)] * xi(c, k) * h;
    const bool xtype = k < N, neg = (k % N) < hN;
    const double lo_pos = neg ? 0.0 : -1.0, hi_pos = neg ? 1.0 : 0.0;
    const double lo = std::exp(a * lo_pos), hi = std::exp(a * hi_pos), mid = std::exp(a * 0.5 * (lo_pos + hi_pos));
    if (f == 4) return mid;
    if (xtype) return f == 0 ? lo : (f == 1 ? hi : mid);
    return f == 2 ? lo : (f == 3 ? hi : mid);
  };
  // selection, eq. (def_V_delta)
  std::vector<std::vector<int>> kidx(static_cast<size_t>(cells));
  std::vector<int64_t> off(size_t(cells) + 1, 0);
  for (int64_t c = 0; c < cells; ++c) {
    for (int k = 0; k < K; ++k)
      if (std::exp(-0.5 * std::fabs(xi(c, k)) * T.sT[size_t(c)] * h) > delta) kidx[size_t(c)].push_back(k);
    off[size_t(c) + 1] = off[size_t(c)] + int64_t(kidx[size_t(c)].size());
  }
  const int64_t nk = off[size_t(cells)];
  out.n_kept = nk;
  out.n_full = cells * K;
  std::vector<int> kpos(size_t(cells) * K, -1);  // position of a kept function among its cell's kept ones
  for (int64_t c = 0; c < cells; ++c)
    for (size_t q = 0; q < kidx[size_t(c)].size(); ++q) kpos[size_t(c) * K + kidx[size_t(c)][q]] = int(q);

  // A is emitted row by row with ascending columns (each face's rows in turn; the
  // cells of a face in index order, their kept functions ascending), so it is
  // built in CSR form directly.  Each row of R belongs to one coefficient and
  // is emitted in one piece (kept: the identity; dropped: by the face its
  // function is centred on), so its pieces are recorded and joined in row order.
  HostCsr& A = out.A;
  A.ptr.assign(1, 0);
  std::vector<int64_t> rcol;
  std::vector<double> rval;
  std::vector<int64_t> rbeg(size_t(cells) * K, -1), rlen(size_t(cells) * K, 0);
  auto r_begin = [&](int64_t t) { rbeg[size_t(t)] = int64_t(rcol.size()); };
  auto r_add = [&](int64_t t, int64_t col, double v) {
    rcol.push_back(col);
    rval.push_back(v);
    rlen[size_t(t)] += 1;
  };
  std::vector<double> bvec, r0(size_t(cells) * K, 0.0);
  // kept coefficients pass through the reconstruction unchanged
  for (int64_t c = 0; c < cells; ++c)
    for (size_t q = 0; q < kidx[size_t(c)].size(); ++q)
    {
      const int64_t t = c * K + kidx[size_t(c)][q];
      r_begin(t);
      r_add(t, off[size_t(c)] + int64_t(q), 1.0);
    }
  int64_t row = 0;
  struct Part {
    int64_t cell;
    int face;    // face of the cell the interface is (0 left 1 right 2 bottom 3 top)
    double seq;  // sign of the part in the condition written as (sum) = rhs
  };
  auto face_go = [&](std::vector<Part> parts, const std::vector<int>& dirs, const std::vector<double>& psi_in) {
    const bool boundary = parts.size() == 1;
    const int nr = int(dirs.size());
    std::vector<std::pair<int64_t, int>> kept, dropped;
    for (const Part& p : parts)
      for (int k = p.face * hN; k < (p.face + 1) * hN; ++k)
        (kpos[size_t(p.cell) * K + k] >= 0 ? kept : dropped).push_back({p.cell, k});
    const int nkf = int(kept.size()), ndf = int(dropped.size());
    RTE_REQUIRE(nkf + ndf == nr, RTE_EINVAL, "ATFPS: face basis does not match the face's directions");
    std::vector<double> H(size_t(nr) * nr, 0.0);
    if (nkf > 0) {
      std::vector<double> Lk(size_t(nr) * nkf), Q, R;
      for (int r = 0; r < nr; ++r)
        for (int q = 0; q < nkf; ++q) Lk[size_t(r) * nkf + q] = Lval(kept[size_t(q)].first, dirs[size_t(r)], kept[size_t(q)].second);
      householder_qr(nr, nkf, Lk, Q, R);
      maxnorm_columns(nr, nkf, Q, true);
      for (int r = 0; r < nr; ++r)
        for (int q = 0; q < nkf; ++q) H[size_t(r) * nr + q] = Q[size_t(r) * nkf + q];
    }
    if (ndf > 0) {
      std::vector<double> Ld(size_t(nr) * ndf);
      for (int r = 0; r < nr; ++r)
        for (int q = 0; q < ndf; ++q) Ld[size_t(r) * ndf + q] = Lval(dropped[size_t(q)].first, dirs[size_t(r)], dropped[size_t(q)].second);
      maxnorm_columns(nr, ndf, Ld, false);
      for (int r = 0; r < nr; ++r)
        for (int q = 0; q < ndf; ++q) H[size_t(r) * nr + nkf + q] = Ld[size_t(r) * ndf + q];
    }
    const std::vector<double> Hi = lu_inverse(nr, H);
    // right-hand side vector of the full condition (before projection)
    std::vector<double> rhs(size_t(nr), 0.0);
    for (const Part& p : parts)
      for (int r = 0; r < nr; ++r) rhs[size_t(r)] -= p.seq * T.chis[size_t(p.cell)];
    if (boundary)
      for (int r = 0; r < nr; ++r) rhs[size_t(r)] += psi_in[size_t(r)];
    // compressed rows: projections onto the kept basis vectors
    for (int p = 0; p < nkf; ++p) {
      for (const Part& pt : parts) {
        const std::vector<int>& kc = kidx[size_t(pt.cell)];
        for (size_t q = 0; q < kc.size(); ++q) {
          const int k = kc[q];
          const double e = efac(pt.cell, k, pt.face);
          double v = 0;
          for (int r = 0; r < nr; ++r) v += Hi[size_t(p) * nr + r] * Lval(pt.cell, dirs[size_t(r)], k);
          A.col.push_back(off[size_t(pt.cell)] + int64_t(q));
          A.val.push_back(pt.seq * v * e);
        }
      }
      A.ptr.push_back(int64_t(A.col.size()));
      double bv = 0;
      for (int r = 0; r < nr; ++r) bv += Hi[size_t(p) * nr + r] * rhs[size_t(r)];
      bvec.push_back(bv);
    }
    row += nkf;
    // layer reconstruction of the dropped coefficients centred on this face
    for (int q = 0; q < ndf; ++q) {
      const int pq = nkf + q;
      const int64_t tgt = dropped[size_t(q)].first * K + dropped[size_t(q)].second;
      r_begin(tgt);
      // interior: sign +1 on the other cell's smooth values, -1 on its own; boundary:
      // the inflow data minus the cell's smooth values
      for (const Part& pt : parts) {
        const double s = boundary ? -1.0 : (pt.cell == dropped[size_t(q)].first ? -1.0 : 1.0);
        const std::vector<int>& kc = kidx[size_t(pt.cell)];
        for (size_t qq = 0; qq < kc.size(); ++qq) {
          const int k = kc[qq];
          double v = 0;
          for (int r = 0; r < nr; ++r) v += Hi[size_t(pq) * nr + r] * Lval(pt.cell, dirs[size_t(r)], k);
          r_add(tgt, off[size_t(pt.cell)] + int64_t(qq), s * v * efac(pt.cell, k, pt.face));
        }
        double cs = 0;
        for (int r = 0; r < nr; ++r) cs += Hi[size_t(pq) * nr + r];
        r0[size_t(tgt)] += s * cs * T.chis[size_t(pt.cell)];
      }
      if (boundary) {
        double v = 0;
        for (int r = 0; r < nr; ++r) v += Hi[size_t(pq) * nr + r] * psi_in[size_t(r)];
        r0[size_t(tgt)] += v;
      }
    }
  };
  // inflow data at a boundary face, from the TFPS right-hand side rows:
  // b = Psi - chi^s of the cell the face belongs to
  std::vector<int> all(static_cast<size_t>(N));
  for (int m = 0; m < N; ++m) all[size_t(m)] = m;
  auto incoming = [&](bool xface, bool lower) {
    std::vector<int> d;
    for (int m = 0; m < N; ++m) {
      const double u = xface ? T.ux[size_t(m)] : T.uy[size_t(m)];
      if (lower ? u > 0 : u < 0) d.push_back(m);
    }
    return d;
  };
  const std::vector<int> in_x0 = incoming(true, true), in_x1 = incoming(true, false);
  const std::vector<int> in_y0 = incoming(false, true), in_y1 = incoming(false, false);
  auto inflow = [&](const std::vector<int>& d, int64_t brow_cell, int blk, int64_t chis_cell) {
    std::vector<double> v(d.size());
    for (size_t r = 0; r < d.size(); ++r)
      v[r] = T.b[size_t(brow_cell) * K + size_t(blk) * N + d[r]] + T.chis[size_t(chis_cell)];
    return v;
  };
  for (int j = 0; j < I; ++j)
    for (int i = 0; i <= I; ++i) {
      if (i == 0) {
        const int64_t c = int64_t(j) * I;
        face_go({{c, 0, 1.0}}, in_x0, inflow(in_x0, c, 0, c));
      } else if (i == I) {
        const int64_t c = int64_t(j) * I + I - 1;
        face_go({{c, 1, 1.0}}, in_x1, inflow(in_x1, int64_t(j) * I, 0, c));
      } else {
        const int64_t cm = int64_t(j) * I + i - 1, cp = cm + 1;
        face_go({{cm, 1, 1.0}, {cp, 0, -1.0}}, all, {});
      }
    }
  for (int i = 0; i < I; ++i)
    for (int j = 0; j <= I; ++j) {
      if (j == 0) {
        const int64_t c = i;
        face_go({{c, 2, 1.0}}, in_y0, inflow(in_y0, c, 1, c));
      } else if (j == I) {
        const int64_t c = int64_t(I - 1) * I + i;
        face_go({{c, 3, 1.0}}, in_y1, inflow(in_y1, int64_t(i), 1, c));
      } else {
        const int64_t cm = int64_t(j - 1) * I + i, cp = cm + I;
        face_go({{cm, 3, 1.0}, {cp, 2, -1.0}}, all, {});
      }
    }
  RTE_REQUIRE(row == nk, RTE_EINVAL, "ATFPS: compressed system is not square");
  out.n_rows = row;
  A.nrows = row;
  A.ncols = nk;
  out.b = std::move(bvec);
  {
    HostCsr& R = out.R;
    R.nrows = cells * K;
    R.ncols = nk;
    R.ptr.assign(1, 0);
    R.col.reserve(rcol.size());
    R.val.reserve(rval.size());
    for (int64_t t = 0; t < cells * K; ++t) {
      RTE_REQUIRE(rbeg[size_t(t)] >= 0, RTE_EINVAL, "ATFPS: a coefficient without a reconstruction row");
      const int64_t b0 = rbeg[size_t(t)];
      R.col.insert(R.col.end(), rcol.begin() + b0, rcol.begin() + b0 + rlen[size_t(t)]);
      R.val.insert(R.val.end(), rval.begin() + b0, rval.begin() + b0 + rlen[size_t(t)]);
      R.ptr.push_back(int64_t(R.col.size()));
    }
  }
  out.r0 = std::move(r0);
  // D_d per cell and M = A_d D_d, c0 = b_d - A_d d0 (psi direction-major [N][cells])
  std::vector<std::vector<double>> Pc(static_cast<size_t>(cells));
  std::vector<double> d0(size_t(nk), 0.0);
  parallel_for(cells, [&](int64_t c) {
    const std::vector<int>& kc = kidx[size_t(c)];
    const int n = int(kc.size());
    if (n == 0) return;
    std::vector<double> Mc(size_t(N) * n);
    for (int m = 0; m < N; ++m)
      for (int q = 0; q < n; ++q) Mc[size_t(m) * n + q] = Lval(c, m, kc[size_t(q)]) * efac(c, kc[size_t(q)], 4);
    Pc[size_t(c)] = pseudo_inverse(N, n, Mc);  // n x N
    for (int q = 0; q < n; ++q) {
      double s = 0;
      for (int m = 0; m < N; ++m) s += Pc[size_t(c)][size_t(q) * N + m];
      d0[size_t(off[size_t(c)] + q)] = -s * T.chis[size_t(c)];
    }
  });
  // M row r = sum over A's entries (r, col) of A_{r,col} times row q of its cell's D: a row
  // touches the directions of at most the two cells of its face, accumulated densely per
  // cell (N values each) and stored once
  HostCsr& M = out.M;
  M.nrows = row;
  M.ncols = int64_t(N) * cells;
  out.c0 = out.b;
  // the cell of kept column col
  auto cell_of = [&](int64_t col) { return int64_t(std::upper_bound(off.begin(), off.end(), col) - off.begin()) - 1; };
  // pass 1: N entries per distinct cell of each row (A's columns ascend, so its cells do)
  M.ptr.assign(size_t(row) + 1, 0);
  parallel_for(row, [&](int64_t r) {
    int64_t nc = 0, last = -1;
    for (int64_t e = out.A.ptr[size_t(r)]; e < out.A.ptr[size_t(r) + 1]; ++e) {
      const int64_t c = cell_of(out.A.col[size_t(e)]);
      if (c != last) {
        ++nc;
        last = c;
      }
    }
    M.ptr[size_t(r) + 1] = nc * N;
  });
  for (int64_t r = 0; r < row; ++r) M.ptr[size_t(r) + 1] += M.ptr[size_t(r)];
  M.col.assign(size_t(M.ptr[size_t(row)]), 0);
  M.val.assign(size_t(M.ptr[size_t(row)]), 0.0);
  // pass 2: M row r = sum over A's entries (r, col) of A_{r,col} times row q of its cell's
  // D, accumulated densely per cell; columns m cells + c, direction-major, cells ascending
  parallel_for(row, [&](int64_t r) {
    int64_t rc[2] = {-1, -1};
    int nc = 0;
    std::vector<double> acc(size_t(2) * N, 0.0);
    double c0r = out.b[size_t(r)];
    for (int64_t e = out.A.ptr[size_t(r)]; e < out.A.ptr[size_t(r) + 1]; ++e) {
      const int64_t col = out.A.col[size_t(e)];
      const double a = out.A.val[size_t(e)];
      c0r -= a * d0[size_t(col)];
      const int64_t c = cell_of(col);
      if (nc == 0 || rc[nc - 1] != c) {
        RTE_REQUIRE(nc < 2, RTE_EINVAL, "ATFPS: a compressed row spans more than two cells");
        rc[nc++] = c;
      }
      double* ac = acc.data() + size_t(nc - 1) * N;
      const double* prow = Pc[size_t(c)].data() + size_t(col - off[size_t(c)]) * N;
      for (int m = 0; m < N; ++m) ac[m] += a * prow[m];
    }
    out.c0[size_t(r)] = c0r;
    int64_t w = M.ptr[size_t(r)];
    for (int m = 0; m < N; ++m)
      for (int k = 0; k < nc; ++k) {
        M.col[size_t(w)] = int64_t(m) * cells + rc[k];
        M.val[size_t(w)] = acc[size_t(k) * N + size_t(m)];
        ++w;
      }
  });
  return out;
}

}  // namespace rte

// Host-only eigen-decomposition of a real symmetric matrix (FP64): Householder
// reduction to tridiagonal form followed by the implicit-shift QL iteration
// (Golub & Van Loan, Matrix Computations, secs. 8.3.1 and 8.3.3), with the
// orthogonal transforms accumulated.  The QL loop takes its steps in the order
// of the published EISPACK routine imtql2 (Bowdler, Martin, Reinsch and
// Wilkinson, Numer. Math. 12, 1968; also "tqli" in Numerical Recipes): the
// shift from the leading 2x2 block, the chase of rotations from the bottom of
// the unreduced block upwards, and the deflation when a rotation radius is 0.  Used for the Gram matrix of a kernel set
// (up to 1024 rows).  The accumulated transform is kept transposed (row i holds
// column i of Q), so every Householder update and every QL rotation runs over
// contiguous rows.
#pragma once

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>
#include <vector>

namespace rf {

// A: n x n symmetric, row-major (only read).  On return w holds the
// eigenvalues in descending order and V (row-major n x n) the matching
// orthonormal eigenvectors as columns: A = V diag(w) V^T.
inline void sym_eig(const std::vector<double>& A_in, int n, std::vector<double>& w, std::vector<double>& V) {
  std::vector<double> A(A_in);
  auto a = [&](int i, int j) -> double& { return A[size_t(i) * n + j]; };
  // Qt: row j is column j of the accumulated orthogonal transform Q
  std::vector<double> Qt(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) Qt[size_t(i) * n + i] = 1.0;
  auto qrow = [&](int j) -> double* { return Qt.data() + size_t(j) * n; };
  std::vector<double> v(n), p(n), wv(n), sq(n);
  // Householder: zero column k below the subdiagonal, for k = 0 .. n-3
  for (int k = 0; k + 2 < n; ++k) {
    double sig = 0.0;
    for (int i = k + 1; i < n; ++i) sig += a(i, k) * a(i, k);
    const double nx = std::sqrt(sig);
    if (nx == 0.0) continue;
    const double x0 = a(k + 1, k);
    const double alpha = x0 > 0 ? -nx : nx;
    // v = x - alpha e1, normalised
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) {
      v[i] = a(i, k) - (i == k + 1 ? alpha : 0.0);
      vn += v[i] * v[i];
    }
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = k + 1; i < n; ++i) v[i] /= vn;
    // trailing block: A <- H A H = A - 2 v w^T - 2 w v^T, w = A v - (v^T A v) v
    double beta = 0.0;
    for (int i = k + 1; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += a(i, j) * v[j];
      p[i] = s;
      beta += v[i] * s;
    }
    for (int i = k + 1; i < n; ++i) wv[i] = p[i] - beta * v[i];
    for (int i = k + 1; i < n; ++i)
      for (int j = k + 1; j < n; ++j) a(i, j) -= 2.0 * (v[i] * wv[j] + wv[i] * v[j]);
    a(k + 1, k) = a(k, k + 1) = alpha;
    for (int i = k + 2; i < n; ++i) a(i, k) = a(k, i) = 0.0;
    // Q <- Q H: column j of Q loses 2 v[j] (Q v), Q v = sum_j v[j] (column j)
    std::fill(sq.begin(), sq.end(), 0.0);
    for (int j = k + 1; j < n; ++j) {
      const double* qj = qrow(j);
      const double vj = v[j];
      for (int r = 0; r < n; ++r) sq[r] += vj * qj[r];
    }
    for (int j = k + 1; j < n; ++j) {
      double* qj = qrow(j);
      const double f = 2.0 * v[j];
      for (int r = 0; r < n; ++r) qj[r] -= f * sq[r];
    }
  }
  // tridiagonal: diagonal d, off-diagonal e[i] = T(i, i + 1), e[n-1] = 0
  std::vector<double> d(n), e(n, 0.0);
  for (int i = 0; i < n; ++i) d[i] = a(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = a(i, i + 1);
  const double eps = 2.220446049250313e-16;
  // an off-diagonal element is negligible against its neighbours or against
  // the whole matrix (eigenvalues below eps |A| are rounding noise anyway)
  double anorm = 0.0;
  for (int i = 0; i < n; ++i) anorm = std::max(anorm, std::fabs(d[i]) + std::fabs(e[i]) + (i ? std::fabs(e[i - 1]) : 0.0));
  const double floor_abs = eps * anorm;
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m + 1 < n; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd || std::fabs(e[m]) <= floor_abs) break;
      }
      if (m == l) break;
      if (iter > 80) throw std::runtime_error("sym_eig: QL iteration did not converge");
      // Wilkinson-type shift from the leading 2x2 block, then chase the bulge
      // from the bottom of the unreduced block [l, m] up to l with rotations
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1.0, c = 1.0, pp = 0.0;
      bool deflated = false;
      for (int i = m - 1; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= pp;
          e[m] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        double* qi = qrow(i);                 // rotate eigenvector columns i, i + 1
        double* qi1 = qrow(i + 1);
        for (int k = 0; k < n; ++k) {
          const double a0 = qi[k], a1 = qi1[k];
          qi1[k] = s * a0 + c * a1;
          qi[k] = c * a0 - s * a1;
        }
      }
      if (deflated) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] > d[y]; });
  w.resize(n);
  V.assign(size_t(n) * n, 0.0);
  for (int c2 = 0; c2 < n; ++c2) {
    w[c2] = d[idx[c2]];
    const double* qc = qrow(idx[c2]);
    for (int k = 0; k < n; ++k) V[size_t(k) * n + c2] = qc[k];
  }
}

}  // namespace rf

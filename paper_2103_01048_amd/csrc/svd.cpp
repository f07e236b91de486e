// One-sided (Hestenes) Jacobi SVD in FP64 and the truncated-SVD
// pseudo-inverse used to solve the KIFMM matching equations (Methods, Fast
// multipole method: the equivalent densities are found by matching
// check-surface potentials and solving the resulting linear systems).
//
// Column pairs are rotated until every pair is orthogonal to working
// precision; the column norms are then the singular values.  The
// pseudo-inverse keeps singular values above tau * s_max.
#include <algorithm>
#include <cmath>
#include <vector>

namespace fmm {

// A: m x n row-major (m >= n).  Returns U (m x n, row-major), s (n), V (n x n,
// row-major) with A = U diag(s) V^T, s unsorted.
static void jacobi_svd(int m, int n, const double *A, std::vector<double> &U,
                       std::vector<double> &s, std::vector<double> &V) {
  // work column-major for contiguous column access
  std::vector<double> a((size_t)m * n), v((size_t)n * n, 0.0);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) a[(size_t)j * m + i] = A[(size_t)i * n + j];
  for (int j = 0; j < n; ++j) v[(size_t)j * n + j] = 1.0;
  std::vector<double> nrm(n);
  for (int j = 0; j < n; ++j) {
    double t = 0;
    const double *c = &a[(size_t)j * m];
    for (int i = 0; i < m; ++i) t += c[i] * c[i];
    nrm[j] = t;
  }
  const double eps = 1e-15;
  for (int sweep = 0; sweep < 60; ++sweep) {
    int rotated = 0;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double *cp = &a[(size_t)p * m], *cq = &a[(size_t)q * m];
        double alpha = nrm[p], beta = nrm[q], gamma = 0;
        for (int i = 0; i < m; ++i) gamma += cp[i] * cq[i];
        if (std::fabs(gamma) <= eps * std::sqrt(alpha * beta) || gamma == 0.0) continue;
        ++rotated;
        double zeta = (beta - alpha) / (2.0 * gamma);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        double np = 0, nq = 0;
        for (int i = 0; i < m; ++i) {
          double x = cp[i], y = cq[i];
          double xn = c * x - sn * y, yn = sn * x + c * y;
          cp[i] = xn;
          cq[i] = yn;
          np += xn * xn;
          nq += yn * yn;
        }
        nrm[p] = np;
        nrm[q] = nq;
        double *vp = &v[(size_t)p * n], *vq = &v[(size_t)q * n];
        for (int i = 0; i < n; ++i) {
          double x = vp[i], y = vq[i];
          vp[i] = c * x - sn * y;
          vq[i] = sn * x + c * y;
        }
      }
    }
    if (!rotated) break;
  }
  s.assign(n, 0.0);
  U.assign((size_t)m * n, 0.0);
  V.assign((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double t = 0;
    const double *c = &a[(size_t)j * m];
    for (int i = 0; i < m; ++i) t += c[i] * c[i];
    s[j] = std::sqrt(t);
    for (int i = 0; i < m; ++i) U[(size_t)i * n + j] = s[j] > 0 ? c[i] / s[j] : 0.0;
    for (int i = 0; i < n; ++i) V[(size_t)i * n + j] = v[(size_t)j * n + i];
  }
}

// Truncated SVD factors of A (n x n): singular values above tau * s_max,
// sorted in decreasing order, are kept (rank r).  UT (n x n, row-major) gets
// U^T in its first r rows and zeros below; VS (n x n, row-major) gets
// V diag(1/s) in its first r columns and zeros to the right, so that
// pinv(A) = VS * UT.  Returns r.
int tsvd_factors(int n, const double *A, double tau, double *UT, double *VS) {
  std::vector<double> U, s, V;
  jacobi_svd(n, n, A, U, s, V);
  std::vector<int> order(n);
  for (int j = 0; j < n; ++j) order[j] = j;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return s[a] > s[b]; });
  const double smax = n ? s[order[0]] : 0.0;
  int r = 0;
  while (r < n && s[order[r]] > tau * smax) ++r;
  std::fill(UT, UT + (size_t)n * n, 0.0);
  std::fill(VS, VS + (size_t)n * n, 0.0);
  for (int k = 0; k < r; ++k) {
    const int j = order[k];
    for (int i = 0; i < n; ++i) {
      UT[(size_t)k * n + i] = U[(size_t)i * n + j];
      VS[(size_t)i * n + k] = V[(size_t)i * n + j] / s[j];
    }
  }
  return r;
}

// out (n x n row-major) = pinv(A) with singular values <= tau * s_max dropped.
void pinv_tsvd(int n, const double *A, double tau, double *out) {
  std::vector<double> U, s, V;
  jacobi_svd(n, n, A, U, s, V);
  double smax = 0;
  for (double x : s) smax = std::max(smax, x);
  std::vector<double> sinv(n, 0.0);
  for (int j = 0; j < n; ++j)
    if (s[j] > tau * smax) sinv[j] = 1.0 / s[j];
  // out = V diag(sinv) U^T
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      double t = 0;
      for (int j = 0; j < n; ++j) t += V[(size_t)i * n + j] * sinv[j] * U[(size_t)k * n + j];
      out[(size_t)i * n + k] = t;
    }
}

}  // namespace fmm

// One-sided (Hestenes) Jacobi SVD in FP64 and the truncated-SVD
// pseudo-inverse used to solve the KIFMM matching equations (Methods, Fast
// multipole method: the equivalent densities are found by matching
// check-surface potentials and solving the resulting linear systems).
//
// Column pairs are rotated until every pair is orthogonal to working
// precision; the column norms are then the singular values.  The
// pseudo-inverse keeps singular values above tau * s_max.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

namespace fmm {

// Threads of one SVD meet at a barrier after every round of rotations.
struct SpinBarrier {
  explicit SpinBarrier(int n) : n_(n) {}
  void wait() {
    const int g = gen_.load(std::memory_order_acquire);
    if (count_.fetch_add(1, std::memory_order_acq_rel) + 1 == n_) {
      count_.store(0, std::memory_order_relaxed);
      gen_.fetch_add(1, std::memory_order_acq_rel);
    } else {
      while (gen_.load(std::memory_order_acquire) == g) std::this_thread::yield();
    }
  }
  std::atomic<int> count_{0}, gen_{0};
  const int n_;
};

// A: m x n row-major (m >= n).  Returns U (m x n, row-major), s (n), V (n x n,
// row-major) with A = U diag(s) V^T, s unsorted.  Each sweep visits every
// column pair once in the round-robin order (n - 1 rounds of disjoint pairs,
// a dummy column when n is odd); the pairs of a round are independent and
// are shared by `nthreads` threads, each pair rotated by the same arithmetic
// whichever thread takes it, so the result does not depend on the thread
// count.
static void jacobi_svd(int m, int n, const double *A, std::vector<double> &U,
                       std::vector<double> &s, std::vector<double> &V, int nthreads) {
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
  const int N = n + (n & 1);  // with a dummy column when n is odd
  auto rotate = [&](int p, int q) -> int {
    double *cp = &a[(size_t)p * m], *cq = &a[(size_t)q * m];
    const double alpha = nrm[p], beta = nrm[q];
    double gamma = 0;
    for (int i = 0; i < m; ++i) gamma += cp[i] * cq[i];
    if (std::fabs(gamma) <= eps * std::sqrt(alpha * beta) || gamma == 0.0) return 0;
    const double zeta = (beta - alpha) / (2.0 * gamma);
    const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
    double np = 0, nq = 0;
    for (int i = 0; i < m; ++i) {
      const double x = cp[i], y = cq[i];
      const double xn = c * x - sn * y, yn = sn * x + c * y;
      cp[i] = xn;
      cq[i] = yn;
      np += xn * xn;
      nq += yn * yn;
    }
    nrm[p] = np;
    nrm[q] = nq;
    double *vp = &v[(size_t)p * n], *vq = &v[(size_t)q * n];
    for (int i = 0; i < n; ++i) {
      const double x = vp[i], y = vq[i];
      vp[i] = c * x - sn * y;
      vq[i] = sn * x + c * y;
    }
    return 1;
  };
  // pair k of round r (circle method over N columns)
  auto pair_of = [&](int r, int k, int &p, int &q) {
    int x = (r + k) % (N - 1), y = (r - k + N - 1) % (N - 1);
    if (k == 0) y = N - 1;
    p = std::min(x, y);
    q = std::max(x, y);
  };
  const int nth = std::max(1, std::min(nthreads, N / 2));
  SpinBarrier bar(nth);
  std::vector<int> rot(nth, 0);
  std::atomic<bool> done{false};
  auto worker = [&](int tid) {
    for (int sweep = 0; sweep < 60; ++sweep) {
      rot[tid] = 0;
      for (int r = 0; r < N - 1; ++r) {
        for (int k = tid; k < N / 2; k += nth) {
          int p, q;
          pair_of(r, k, p, q);
          if (q < n) rot[tid] += rotate(p, q);
        }
        bar.wait();
      }
      if (tid == 0) {
        int total = 0;
        for (int t = 0; t < nth; ++t) total += rot[t];
        done.store(total == 0, std::memory_order_release);
      }
      bar.wait();
      if (done.load(std::memory_order_acquire)) break;
      bar.wait();  // every thread has read `done` before the next sweep resets its count
    }
  };
  if (N >= 2) {
    std::vector<std::thread> th;
    for (int t = 1; t < nth; ++t) th.emplace_back(worker, t);
    worker(0);
    for (auto &t : th) t.join();
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
int tsvd_factors(int n, const double *A, double tau, double *UT, double *VS, int nthreads) {
  std::vector<double> U, s, V;
  jacobi_svd(n, n, A, U, s, V, nthreads);
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

// Low-rank split of A (rows x cols, row-major): with A = U S V^T and the k
// singular values above tau * s_max kept (decreasing order),
// L = U_k S_k^{1/2} (rows x k, row-major, leading dimension ldl) and
// R = S_k^{1/2} V_k^T (k x cols, row-major, leading dimension ldr), so that
// A ~ L R.  Returns k (0 for a zero matrix).
int tsvd_split(int rows, int cols, const double *A, double tau, double *L, int ldl, double *R, int ldr) {
  // the one-sided Jacobi SVD wants at least as many rows as columns: work on
  // the transpose when A is wide
  const bool tr = rows < cols;
  const int m = tr ? cols : rows, n = tr ? rows : cols;
  std::vector<double> B((size_t)m * n);
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) {
      if (tr) B[(size_t)j * n + i] = A[(size_t)i * cols + j];
      else B[(size_t)i * n + j] = A[(size_t)i * cols + j];
    }
  std::vector<double> U, s, V;
  jacobi_svd(m, n, B.data(), U, s, V, 1);
  std::vector<int> order(n);
  for (int j = 0; j < n; ++j) order[j] = j;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return s[a] > s[b]; });
  const double smax = n ? s[order[0]] : 0.0;
  int k = 0;
  while (k < n && s[order[k]] > tau * smax && s[order[k]] > 0.0) ++k;
  // B = U S V^T (m x n); A = B or B^T
  for (int c = 0; c < k; ++c) {
    const int j = order[c];
    const double h = std::sqrt(s[j]);
    for (int i = 0; i < rows; ++i) L[(size_t)i * ldl + c] = h * (tr ? V[(size_t)i * n + j] : U[(size_t)i * n + j]);
    for (int i = 0; i < cols; ++i) R[(size_t)c * ldr + i] = h * (tr ? U[(size_t)i * n + j] : V[(size_t)i * n + j]);
  }
  return k;
}

// out (n x n row-major) = pinv(A) with singular values <= tau * s_max dropped.
void pinv_tsvd(int n, const double *A, double tau, double *out) {
  std::vector<double> U, s, V;
  jacobi_svd(n, n, A, U, s, V, 1);
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

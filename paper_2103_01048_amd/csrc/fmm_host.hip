// Host planner of the MI355X FMM library: argument checks, octree and
// interaction lists, FP64 operator precompute, task lists, and the C ABI
// entry points fmm_setup / fmm_eval / fmm_info / fmm_get_tree / fmm_free.
//
// Tree (Methods, Fast multipole method: an enclosing cube subdivided until
// each leaf holds at most a constant number of points):
//   root cube centred on the bounding box, side W = extent * (1 + 2^-20);
//   63-bit Morton keys floor(((x - lo) / W) * 2^21) per axis, interleaved
//   x,y,z; stable sort; a box splits while it holds more than ncrit points
//   (level cap 21); boxes numbered by (level, key).
// Lists of an adaptive tree: U (adjacent leaves), V (the interaction list:
// children of the parent's neighbours not adjacent to the box), W
// (descendants of neighbours not adjacent but with an adjacent parent) and
// X (the transpose of W).
// Operators (the matching equations for upward and downward equivalent
// densities): surfaces of p x p x p grid points on cubes of half-width
// 1.05 h / 2.95 h; check-to-equivalent maps are truncated-SVD
// pseudo-inverses computed in FP64; M2M, L2L and M2L are kernel matrices
// between surfaces (M2M composed with the parent's pseudo-inverse).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <atomic>
#include <array>
#include <map>
#include <mutex>
#include <thread>

#include "fmm_internal.h"

namespace fmm {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

int device_bbox(const double *xyz, int64_t n, hipStream_t s, double mn[3], double mx[3], bool *finite,
                uint64_t *hash);
int device_morton_sort(const double *xyz, int64_t n, const std::vector<int64_t> &off, const std::vector<double> &lo,
                       double W, hipStream_t s, std::vector<int64_t> &keys_out, std::vector<int64_t> &perm_out,
                       uint64_t **keys_dev);
int device_tree(fmm_plan *P, const uint64_t *d_keys, hipStream_t s, double *ms_tree, double *ms_lists);
int device_gather_leaves(const double *xyz, const int32_t *perm, const std::vector<int64_t> &lb,
                         const std::vector<int64_t> &le, const std::vector<double> &lsh, int prec, void *pts,
                         hipStream_t s);
int eval_dispatch(fmm_plan *P, const void *q, int nrhs, void *pot, void *grad, hipStream_t s);
int eval_pair_dispatch(fmm_plan *A, fmm_plan *B, const void *q, int nrhs, void *pot_a, void *grad_a, void *pot_b,
                       void *grad_b, hipStream_t s);
int eval_pair_md_dispatch(fmm_plan *A, fmm_plan *B, const void *q, const void *dip, double ca, double cb, void *pot_a,
                          void *grad_a, void *pot_b, void *grad_b, hipStream_t s);
int adjoint_combine(fmm_plan *P, int nrhs, const void *q, const void *gbar, const void *gphi, const void *gpsi,
                    void *dx, hipStream_t s);

static int dev_alloc(fmm_plan *P, void **ptr, size_t bytes) {
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    set_error("hipMalloc(" + std::to_string(bytes) + " bytes): " + hipGetErrorString(e));
    *ptr = nullptr;
    return FMM_ENOMEM;
  }
  (P->alloc_sink ? *P->alloc_sink : P->allocs).push_back(*ptr);
  P->device_bytes += (int64_t)bytes;
  return FMM_OK;
}

// A device copy of `bytes` host bytes owned by plan P (freed by fmm_free);
// with h null, an uninitialised allocation.
int plan_upload(fmm_plan *P, void **ptr, const void *h, size_t bytes) {
  int rc = dev_alloc(P, ptr, bytes);
  if (rc) return rc;
  if (bytes && h) FMM_HIP_TRY(hipMemcpy(*ptr, h, bytes, hipMemcpyHostToDevice));
  return FMM_OK;
}

template <typename V>
static int upload(fmm_plan *P, void **ptr, const std::vector<V> &h) {
  int rc = dev_alloc(P, ptr, h.size() * sizeof(V));
  if (rc) return rc;
  if (!h.empty()) FMM_HIP_TRY(hipMemcpy(*ptr, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
  return FMM_OK;
}

// FP64 host values to the plan's working type.
static int upload_real(fmm_plan *P, void **ptr, const std::vector<double> &h) {
  if (P->precision == FMM_FP64) return upload(P, ptr, h);
  std::vector<float> f(h.begin(), h.end());
  return upload(P, ptr, f);
}

// ---------------------------------------------------------------------------
// Tree
// ---------------------------------------------------------------------------
static inline int64_t interleave3(int64_t x, int64_t y, int64_t z, int l) {
  int64_t k = 0;
  for (int b = 0; b < l; ++b) {
    k |= ((x >> b) & 1) << (3 * b + 2);
    k |= ((y >> b) & 1) << (3 * b + 1);
    k |= ((z >> b) & 1) << (3 * b);
  }
  return k;
}

struct Lookup {
  // per level: the prefixes of the level's boxes (ordered by molecule, then
  // key) and, per molecule, its range within the level
  const fmm_plan *P;
  std::vector<std::vector<int64_t>> pre;
  std::vector<std::vector<std::pair<int64_t, int64_t>>> rng;
  explicit Lookup(const fmm_plan *p) : P(p) {
    const int nl = (int)P->level_begin.size() - 1;
    const int nmol = (int)P->mol_off.size() - 1;
    pre.resize(nl);
    rng.assign(nl, std::vector<std::pair<int64_t, int64_t>>(nmol, {0, 0}));
    for (int l = 0; l < nl; ++l)
      for (int64_t b = P->level_begin[l]; b < P->level_begin[l + 1]; ++b) {
        const int64_t i = (int64_t)pre[l].size();
        pre[l].push_back(interleave3(P->anchor[3 * b], P->anchor[3 * b + 1], P->anchor[3 * b + 2], l));
        auto &r = rng[l][P->mol[b]];
        if (r.second == r.first) r = {i, i + 1};
        else r.second = i + 1;
      }
  }
  int64_t find(int mol, int l, int64_t x, int64_t y, int64_t z) const {
    if (l >= (int)pre.size()) return -1;
    const int64_t side = (int64_t)1 << l;
    if (x < 0 || y < 0 || z < 0 || x >= side || y >= side || z >= side) return -1;
    const int64_t k = interleave3(x, y, z, l);
    const auto r = rng[l][mol];
    auto b0 = pre[l].begin() + r.first, b1 = pre[l].begin() + r.second;
    auto it = std::lower_bound(b0, b1, k);
    if (it == b1 || *it != k) return -1;
    return P->level_begin[l] + (it - pre[l].begin());
  }
};

static bool adjacent(const fmm_plan *P, int64_t a, int64_t b) {
  const int la = P->level[a], lbv = P->level[b];
  const int64_t sa = (int64_t)1 << (MAXLEVEL - la), sb = (int64_t)1 << (MAXLEVEL - lbv);
  for (int d = 0; d < 3; ++d) {
    const int64_t loa = P->anchor[3 * a + d] * sa, lob = P->anchor[3 * b + d] * sb;
    if (loa > lob + sb || lob > loa + sa) return false;
  }
  return true;
}

static void build_lists(fmm_plan *P) {
  const int64_t nb = (int64_t)P->level.size();
  Lookup lk(P);
  std::vector<std::vector<int64_t>> U(nb), V(nb), Wl(nb), X(nb);
  auto children = [&](int64_t b, std::vector<int64_t> &out) {
    for (int c = 0; c < P->nchild[b]; ++c) out.push_back(P->child_begin[b] + c);
  };
  for (int64_t b = 0; b < nb; ++b) {
    const int l = P->level[b];
    const int64_t ax = P->anchor[3 * b], ay = P->anchor[3 * b + 1], az = P->anchor[3 * b + 2];
    if (l >= 2) {
      const int64_t p = P->parent[b];
      const int64_t px = P->anchor[3 * p], py = P->anchor[3 * p + 1], pz = P->anchor[3 * p + 2];
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            const int64_t c = lk.find(P->mol[b], l - 1, px + dx, py + dy, pz + dz);
            if (c < 0) continue;
            for (int k = 0; k < P->nchild[c]; ++k) {
              const int64_t ch = P->child_begin[c] + k;
              if (!adjacent(P, ch, b)) V[b].push_back(ch);
            }
          }
      std::sort(V[b].begin(), V[b].end());
    }
    if (P->nchild[b] != 0) continue;
    std::vector<int64_t> uu, ww, stack;
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          int64_t cx = ax + dx, cy = ay + dy, cz = az + dz;
          const int64_t side = (int64_t)1 << l;
          if (cx < 0 || cy < 0 || cz < 0 || cx >= side || cy >= side || cz >= side) continue;
          int ll = l;
          int64_t box = -1;
          while (ll >= 0) {
            box = lk.find(P->mol[b], ll, cx, cy, cz);
            if (box >= 0) break;
            --ll;
            cx >>= 1; cy >>= 1; cz >>= 1;
          }
          if (box < 0) continue;
          if (P->nchild[box] == 0) {
            uu.push_back(box);
          } else if (ll == l) {
            stack.clear();
            children(box, stack);
            while (!stack.empty()) {
              const int64_t d = stack.back();
              stack.pop_back();
              if (adjacent(P, d, b)) {
                if (P->nchild[d] == 0) uu.push_back(d);
                else children(d, stack);
              } else {
                ww.push_back(d);
              }
            }
          }
        }
    std::sort(uu.begin(), uu.end());
    uu.erase(std::unique(uu.begin(), uu.end()), uu.end());
    std::sort(ww.begin(), ww.end());
    ww.erase(std::unique(ww.begin(), ww.end()), ww.end());
    U[b] = uu;
    Wl[b] = ww;
  }
  for (int64_t b = 0; b < nb; ++b)
    for (int64_t a : Wl[b]) X[a].push_back(b);
  std::vector<std::vector<int64_t>> *L[4] = {&U, &V, &Wl, &X};
  for (int k = 0; k < 4; ++k) {
    P->loff[k].assign(nb + 1, 0);
    P->lidx[k].clear();
    for (int64_t b = 0; b < nb; ++b) {
      P->loff[k][b + 1] = P->loff[k][b] + (int64_t)(*L[k])[b].size();
      P->lidx[k].insert(P->lidx[k].end(), (*L[k])[b].begin(), (*L[k])[b].end());
    }
  }
}

// ---------------------------------------------------------------------------
// Operators
// ---------------------------------------------------------------------------
static std::vector<double> surface_grid(int p) {
  std::vector<double> g;
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j)
      for (int k = 0; k < p; ++k)
        if (std::min(i, std::min(j, k)) == 0 || std::max(i, std::max(j, k)) == p - 1) {
          g.push_back(2.0 * i / (p - 1) - 1.0);
          g.push_back(2.0 * j / (p - 1) - 1.0);
          g.push_back(2.0 * k / (p - 1) - 1.0);
        }
  return g;
}

// K[i][j] = g(|x_i - y_j|) without 1/(4 pi); x_i = cx + ax*grid_i, y_j = cy + ay*grid_j
static void kernel_matrix(const std::vector<double> &grid, int n, const double cx[3], double ax, const double cy[3],
                          double ay, int yuk, double kappa, double *out, int ldo) {
  for (int i = 0; i < n; ++i) {
    const double x0 = cx[0] + ax * grid[3 * i], x1 = cx[1] + ax * grid[3 * i + 1], x2 = cx[2] + ax * grid[3 * i + 2];
    for (int j = 0; j < n; ++j) {
      const double d0 = x0 - (cy[0] + ay * grid[3 * j]);
      const double d1 = x1 - (cy[1] + ay * grid[3 * j + 1]);
      const double d2 = x2 - (cy[2] + ay * grid[3 * j + 2]);
      const double r = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      out[(size_t)i * ldo + j] = r == 0.0 ? 0.0 : (yuk ? std::exp(-kappa * r) / r : 1.0 / r);
    }
  }
}

// C (m x p, ldc) = A (m x k, lda) * B (k x p, ldb)
static void matmul_rect(int m, int k, int p, const double *A, int lda, const double *B, int ldb, double *C, int ldc) {
  std::vector<double> row(p);
  for (int i = 0; i < m; ++i) {
    std::fill(row.begin(), row.end(), 0.0);
    for (int kk = 0; kk < k; ++kk) {
      const double a = A[(size_t)i * lda + kk];
      if (a == 0.0) continue;
      const double *b = B + (size_t)kk * ldb;
      for (int j = 0; j < p; ++j) row[j] += a * b[j];
    }
    std::copy(row.begin(), row.end(), C + (size_t)i * ldc);
  }
}

static void matmul(int n, const double *A, const double *B, int ldb, double *C, int ldc) {
  // C (n x n, ldc) = A (n x n) * B (n x n, ldb)
  std::vector<double> row(n);
  for (int i = 0; i < n; ++i) {
    std::fill(row.begin(), row.end(), 0.0);
    for (int k = 0; k < n; ++k) {
      const double a = A[(size_t)i * n + k];
      const double *b = B + (size_t)k * ldb;
      for (int j = 0; j < n; ++j) row[j] += a * b[j];
    }
    std::copy(row.begin(), row.end(), C + (size_t)i * ldc);
  }
}

template <typename F>
static void parallel_for(int64_t count, F f) {
  unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  if (count <= 1 || nt == 1) { for (int64_t i = 0; i < count; ++i) f(i); return; }
  std::vector<std::thread> th;
  std::atomic<int64_t> next(0);
  for (unsigned t = 0; t < std::min<int64_t>(nt, count); ++t)
    th.emplace_back([&]() { for (int64_t i; (i = next.fetch_add(1)) < count;) f(i); });
  for (auto &t : th) t.join();
}

// Swizzle a dense row-major matrix A (rows x K, lda) into the MFMA fragment
// order used by k_gemm: element [((rb*(K/16) + kq)*64 + lane)*4 + t] holds
// A[rb*16 + slot(lane%16)][(kq*4 + t)*4 + lane/16].
// The 16x16x4 f32 MFMA returns rows 4*(lane/16) + reg of its 16x16 block in
// lane order; the f64 one returns rows lane/16 + 4*reg.  For double, row
// slot s of the block is fed with row 4*(s%4) + s/4, so that both types
// leave four consecutive rows in each lane's four result registers.
template <typename T>
static void swizzle(const double *A, int rows, int cols, int lda, int ld_rows, int Kfull, T *out) {
  const int KQ = Kfull / 16;
  const bool f64 = sizeof(T) == 8;
  for (int rb = 0; rb < ld_rows / 16; ++rb)
    for (int kq = 0; kq < KQ; ++kq)
      for (int lane = 0; lane < 64; ++lane)
        for (int t = 0; t < 4; ++t) {
          const int sl = lane & 15;
          const int i = rb * 16 + (f64 ? 4 * (sl & 3) + (sl >> 2) : sl), k = (kq * 4 + t) * 4 + (lane >> 4);
          const double v = (i < rows && k < cols) ? A[(size_t)i * lda + k] : 0.0;
          out[((size_t)(rb * KQ + kq) * 64 + lane) * 4 + t] = (T)v;
        }
}

static int m2l_code(int ox, int oy, int oz) { return (ox + 3) * 49 + (oy + 3) * 7 + (oz + 3); }

static inline uint16_t bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
static inline float bf16_to_f(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// Split a row-major matrix (rows x cols) into bf16 high and low parts in the
// fragment order of k_gemm_bf3: for row block rb and 32-wide k block kb, 64
// lanes x 8 values of the high part, then 64 x 8 of the low part; lane l
// holds row rb*16 + l%16, k = kb*32 + 8*(l/16) .. +7.
static void swizzle_bf3(const double *A, int rows, int cols, int lda, int ld_rows, int KB, uint16_t *out) {
  for (int rb = 0; rb < ld_rows / 16; ++rb)
    for (int kb = 0; kb < KB; ++kb)
      for (int lane = 0; lane < 64; ++lane)
        for (int e = 0; e < 8; ++e) {
          const int i = rb * 16 + (lane & 15), k = kb * 32 + 8 * (lane >> 4) + e;
          const double v = (i < rows && k < cols) ? A[(size_t)i * lda + k] : 0.0;
          const uint16_t h = bf16_rne((float)v);
          const uint16_t l = bf16_rne((float)(v - (double)bf16_to_f(h)));
          const size_t base = ((size_t)(rb * KB + kb) * 2) * 64 * 8;
          out[base + lane * 8 + e] = h;
          out[base + 64 * 8 + lane * 8 + e] = l;
        }
}

template <typename T>
static int precompute_typed(fmm_plan *P) {
  const int p = P->p, n = P->nsurf, ld = P->ld;
  const int yuk = P->kernel == FMM_YUKAWA;
  const int maxl = (int)P->level_begin.size() - 2;
  // singular values kept above tau * s_max: FP64 1e-11 up to p = 7 and
  // 10^-(p+1) from p = 8 (1e-9 at p = 8: more than an order of magnitude
  // below the expansion error there, about 3e-8, and ranks of 247-262
  // instead of 287-292 of 296); single precision 1e-6 (components below
  // that are at the FP32 rounding level of the data that flows through them)
  const double tau = P->precision == FMM_FP64 ? (p >= 8 ? std::pow(10.0, -(p + 1)) : 1e-11) : 1e-6;
  const std::vector<double> grid = surface_grid(p);
  const double zero[3] = {0, 0, 0};
  auto h_of = [&](int l) { return P->W / (double)(1ll << (l + 1)); };

  std::vector<std::vector<char>> m2l_used(maxl + 1, std::vector<char>(343, 0));
  for (int64_t b = 0; b < (int64_t)P->level.size(); ++b)
    for (int64_t k = P->loff[1][b]; k < P->loff[1][b + 1]; ++k) {
      const int64_t a = P->lidx[1][k];
      const int c = m2l_code((int)(P->anchor[3 * a] - P->anchor[3 * b]), (int)(P->anchor[3 * a + 1] - P->anchor[3 * b + 1]),
                             (int)(P->anchor[3 * a + 2] - P->anchor[3 * b + 2]));
      m2l_used[P->level[b]][c] = 1;
    }
  std::vector<char> has_children(maxl + 1, 0);
  for (int64_t b = 0; b < (int64_t)P->level.size(); ++b)
    if (P->nchild[b]) has_children[P->level[b]] = 1;

  // Geometry levels for which matrices are computed: every level >= 2 for
  // Yukawa; one unit level (half-width 1) for Laplace, whose kernel scales as
  // 1/h, so that level l uses the unit matrices times a power of h_l.
  std::vector<int> glevels;
  if (yuk) for (int l = 2; l <= maxl; ++l) glevels.push_back(l);
  else if (maxl >= 2) glevels.push_back(-1);
  auto gh = [&](int gl) { return gl < 0 ? 1.0 : h_of(gl); };

  // kinds: 0 UT_u, 1 VS_u, 2 UT_d, 3 VS_d, 4 M2M (per octant), 5 L2L, 6 M2L.
  // M2M, L2L and M2L act between singular coordinates of the check
  // potentials (c = U^T chk, equivalent density = V S^-1 c):
  //   M2M_c  = U_u^T(l)   K(parent upward check, child c upward equiv) V_u S_u^-1(l+1)
  //   L2L_c  = U_d^T(l+1) K(child c downward check, parent downward equiv) V_d S_d^-1(l)
  //   M2L_o  = U_d^T(l)   K(downward check, upward equiv at offset o) V_u S_u^-1(l)
  struct Job { int kind, l, oct, code; };
  std::vector<Job> jobs;
  for (int gl : glevels) {
    for (int k = 0; k < 4; ++k) jobs.push_back({k, gl, 0, 0});
    const bool kids = gl < 0 || (gl < maxl && has_children[gl]);
    if (kids) {
      for (int c = 0; c < 8; ++c) jobs.push_back({4, gl, c, 0});
      for (int c = 0; c < 8; ++c) jobs.push_back({5, gl, c, 0});
    }
    for (int code = 0; code < 343; ++code) {
      bool used = false;
      if (gl < 0) { for (int l = 2; l <= maxl; ++l) used |= m2l_used[l][code] != 0; }
      else used = m2l_used[gl][code] != 0;
      if (used) jobs.push_back({6, gl, 0, code});
    }
  }
  // truncated SVD factors of the check-from-equivalent matrices
  std::map<int, std::vector<double>> ut_u, vs_u, ut_d, vs_d;
  std::map<int, int> rk_u, rk_d;
  std::vector<int> svd_levels = glevels;
  if (yuk && maxl >= 2) svd_levels.push_back(maxl + 1);  // never used; keeps l+1 lookups defined
  for (int gl : svd_levels) {
    ut_u[gl].assign((size_t)n * n, 0); vs_u[gl].assign((size_t)n * n, 0);
    ut_d[gl].assign((size_t)n * n, 0); vs_d[gl].assign((size_t)n * n, 0);
    rk_u[gl] = rk_d[gl] = 0;
  }
  {
    std::vector<std::pair<int, int>> pj;
    for (int gl : glevels) { pj.push_back({0, gl}); pj.push_back({1, gl}); }
    std::vector<int> ranks(pj.size());
    // the host threads split between the SVDs that run at once
    const int hw = (int)std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    const int per_svd = std::max(1, hw / (int)std::max<size_t>(1, pj.size()));
    parallel_for((int64_t)pj.size(), [&](int64_t i) {
      const int kind = pj[i].first, gl = pj[i].second;
      const double h = gh(gl);
      std::vector<double> Km((size_t)n * n);
      if (kind == 0) {
        kernel_matrix(grid, n, zero, ALPHA_UC * h, zero, ALPHA_UE * h, yuk, P->kappa, Km.data(), n);
        ranks[i] = tsvd_factors(n, Km.data(), tau, ut_u[gl].data(), vs_u[gl].data(), per_svd);
      } else {
        kernel_matrix(grid, n, zero, ALPHA_DC * h, zero, ALPHA_DE * h, yuk, P->kappa, Km.data(), n);
        ranks[i] = tsvd_factors(n, Km.data(), tau, ut_d[gl].data(), vs_d[gl].data(), per_svd);
      }
    });
    for (size_t i = 0; i < pj.size(); ++i) (pj[i].first == 0 ? rk_u : rk_d)[pj[i].second] = ranks[i];
  }
  auto r16 = [](int r) { return std::max(16, ((r + 15) / 16) * 16); };
  // the child level of a geometry level (Laplace: the unit level itself,
  // with the child factors scaled by 1/2 below)
  auto child_of = [&](int gl) { return gl < 0 ? gl : gl + 1; };
  std::vector<int> id1(jobs.size(), -1), id8(jobs.size(), -1);
  int64_t c1 = 0;
  for (size_t j = 0; j < jobs.size(); ++j) id1[j] = (int)c1++;
  // factored M2L: each M2L job also stores its right factor R (id1 then holds
  // the left factor L); rank per job
  const bool fact = P->tune.m2l_factored != 0;
  std::vector<int> idr(jobs.size(), -1), rankf(jobs.size(), 0);
  if (fact)
    for (size_t j = 0; j < jobs.size(); ++j)
      if (jobs[j].kind == 6) idr[j] = (int)c1++;
  const double tau_f = P->precision == FMM_FP64 ? 1e-11 : 1e-7;
  const size_t m1 = (size_t)ld * ld;
  std::vector<T> pool1(std::max<size_t>(1, c1 * m1));
  // bf16x3 mode: the M2L operators also in split bf16 form (K padded to 32)
  const bool bf3 = P->precision == FMM_FP32_BF16X3;
  const int KB = (ld + 31) / 32;
  const size_t mbf = (size_t)(ld / 16) * KB * 2 * 64 * 8;
  std::vector<int> idbf(jobs.size(), -1), idbfr(jobs.size(), -1);
  int64_t cbf = 0;
  if (bf3)
    for (size_t j = 0; j < jobs.size(); ++j)
      if (jobs[j].kind == 6) {
        idbf[j] = (int)cbf++;
        if (fact) idbfr[j] = (int)cbf++;
      }
  std::vector<uint16_t> poolbf(std::max<size_t>(1, cbf * mbf));
  parallel_for((int64_t)jobs.size(), [&](int64_t j) {
    const Job &jb = jobs[j];
    const double h = gh(jb.l);
    T *dst = pool1.data() + id1[j] * m1;
    switch (jb.kind) {
      case 0: swizzle<T>(ut_u[jb.l].data(), n, n, n, ld, ld, dst); break;
      case 1: swizzle<T>(vs_u[jb.l].data(), n, n, n, ld, ld, dst); break;
      case 2: swizzle<T>(ut_d[jb.l].data(), n, n, n, ld, ld, dst); break;
      case 3: swizzle<T>(vs_d[jb.l].data(), n, n, n, ld, ld, dst); break;
      case 4: {
        // octant c: parent singular coordinates from the child's
        const int cl = child_of(jb.l);
        const int rp = rk_u[jb.l], rc = rk_u[cl];
        const double cs = jb.l < 0 ? 0.5 : 1.0;  // Laplace: child V S^-1 at half the unit size
        const int c = jb.oct;
        std::vector<double> Km((size_t)n * n), KV((size_t)n * rc), M((size_t)rp * rc);
        const double off[3] = {(((c >> 2) & 1) ? 0.5 : -0.5) * h, (((c >> 1) & 1) ? 0.5 : -0.5) * h,
                               ((c & 1) ? 0.5 : -0.5) * h};
        kernel_matrix(grid, n, zero, ALPHA_UC * h, off, ALPHA_UE * h * 0.5, yuk, P->kappa, Km.data(), n);
        matmul_rect(n, n, rc, Km.data(), n, vs_u[cl].data(), n, KV.data(), rc);
        matmul_rect(rp, n, rc, ut_u[jb.l].data(), n, KV.data(), rc, M.data(), rc);
        for (double &v : M) v *= cs;
        swizzle<T>(M.data(), rp, rc, rc, ld, ld, dst);
        break;
      }
      case 5: {
        const int cl = child_of(jb.l);
        const int c = jb.oct;
        const int rp = rk_d[jb.l], rc = rk_d[cl];
        const double off[3] = {(((c >> 2) & 1) ? 0.5 : -0.5) * h, (((c >> 1) & 1) ? 0.5 : -0.5) * h,
                               ((c & 1) ? 0.5 : -0.5) * h};
        std::vector<double> Km((size_t)n * n), KV((size_t)n * rp), M((size_t)rc * rp);
        kernel_matrix(grid, n, off, ALPHA_DC * h * 0.5, zero, ALPHA_DE * h, yuk, P->kappa, Km.data(), n);
        matmul_rect(n, n, rp, Km.data(), n, vs_d[jb.l].data(), n, KV.data(), rp);
        matmul_rect(rc, n, rp, ut_d[cl].data(), n, KV.data(), rp, M.data(), rp);
        swizzle<T>(M.data(), rc, rp, rp, ld, ld, dst);
        break;
      }
      default: {
        const int code = jb.code;
        const double o[3] = {2.0 * h * (code / 49 - 3), 2.0 * h * ((code / 7) % 7 - 3), 2.0 * h * (code % 7 - 3)};
        const int ru = rk_u[jb.l], rd = rk_d[jb.l];
        std::vector<double> Km((size_t)n * n), KV((size_t)n * ru), M((size_t)rd * ru);
        kernel_matrix(grid, n, zero, ALPHA_DC * h, o, ALPHA_UE * h, yuk, P->kappa, Km.data(), n);
        matmul_rect(n, n, ru, Km.data(), n, vs_u[jb.l].data(), n, KV.data(), ru);
        matmul_rect(rd, n, ru, ut_d[jb.l].data(), n, KV.data(), ru, M.data(), ru);
        if (fact) {
          // M ~ L R (rank k): L (rd x k) where the operator was, R (k x ru)
          // in its own slot
          std::vector<double> Lf((size_t)rd * rd, 0.0), Rf((size_t)std::min(rd, ru) * ru, 0.0);
          const int kf = std::max(1, tsvd_split(rd, ru, M.data(), tau_f, Lf.data(), rd, Rf.data(), ru));
          rankf[j] = kf;
          swizzle<T>(Lf.data(), rd, kf, rd, ld, ld, dst);
          swizzle<T>(Rf.data(), kf, ru, ru, ld, ld, pool1.data() + idr[j] * m1);
          if (bf3) {
            swizzle_bf3(Lf.data(), rd, kf, rd, ld, KB, poolbf.data() + idbf[j] * mbf);
            swizzle_bf3(Rf.data(), kf, ru, ru, ld, KB, poolbf.data() + idbfr[j] * mbf);
          }
        } else {
          swizzle<T>(M.data(), rd, ru, ru, ld, ld, dst);
          if (idbf[j] >= 0) swizzle_bf3(M.data(), rd, ru, ru, ld, KB, poolbf.data() + idbf[j] * mbf);
        }
      }
    }
  });
  // per-level matrix ids, ranks and scale factors.  Laplace: K(h) = K(1)/h,
  // so V S^-1 at level l is h_l times the unit factor; M2M, L2L and M2L in
  // singular coordinates are scale-free.
  const int L1 = maxl + 1;
  P->utu_id.assign(L1, -1); P->vsu_id.assign(L1, -1); P->utd_id.assign(L1, -1); P->vsd_id.assign(L1, -1);
  P->rank_u.assign(L1 + 1, 0); P->rank_d.assign(L1 + 1, 0);
  P->m2m_id.assign(L1, std::vector<int>(8, -1));
  P->l2l_id.assign(L1, std::vector<int>(8, -1));
  P->m2l_id.assign(L1, std::vector<int>(343, -1));
  P->m2l_r_id.assign(L1, std::vector<int>(343, -1));
  P->m2l_k.assign(L1, std::vector<int>(343, 0));
  P->vs_alpha.assign(L1, 1); P->k_alpha.assign(L1, 1);
  for (int l = 2; l <= maxl; ++l) {
    const int gl = yuk ? l : -1;
    P->rank_u[l] = rk_u[gl];
    P->rank_d[l] = rk_d[gl];
    P->vs_alpha[l] = yuk ? 1.0 : h_of(l);
  }
  for (size_t j = 0; j < jobs.size(); ++j) {
    const Job &jb = jobs[j];
    for (int l = 2; l <= maxl; ++l) {
      if (jb.l >= 0 && jb.l != l) continue;
      switch (jb.kind) {
        case 0: P->utu_id[l] = id1[j]; break;
        case 1: P->vsu_id[l] = id1[j]; break;
        case 2: P->utd_id[l] = id1[j]; break;
        case 3: P->vsd_id[l] = id1[j]; break;
        case 4: P->m2m_id[l][jb.oct] = id1[j]; break;
        case 5: P->l2l_id[l][jb.oct] = id1[j]; break;
        case 6:
          P->m2l_id[l][jb.code] = bf3 ? idbf[j] : id1[j];
          P->m2l_r_id[l][jb.code] = bf3 ? idbfr[j] : idr[j];
          P->m2l_k[l][jb.code] = rankf[j];
          break;
      }
    }
  }
  P->pool1_count = c1;
  P->m2l_ldt = 0;
  if (fact) {
    int kmax = 1;
    for (size_t j = 0; j < jobs.size(); ++j) kmax = std::max(kmax, rankf[j]);
    P->m2l_ldt = ((kmax + 31) / 32) * 32;
  }
  int rc;
  if ((rc = upload(P, &P->pool1, pool1))) return rc;
  P->bf_kb = KB;
  P->poolbf_count = cbf;
  if (bf3 && (rc = upload(P, &P->pool_bf, poolbf))) return rc;
  // surface grid table (T4)
  std::vector<T> sg((size_t)n * 4);
  for (int i = 0; i < n; ++i) {
    sg[4 * i] = (T)grid[3 * i]; sg[4 * i + 1] = (T)grid[3 * i + 1]; sg[4 * i + 2] = (T)grid[3 * i + 2]; sg[4 * i + 3] = 0;
  }
  if ((rc = upload(P, &P->surf, sg))) return rc;
  // box geometry (T4: centre relative to the root centre, half width)
  const int64_t nb = (int64_t)P->level.size();
  std::vector<T> geom((size_t)nb * 4);
  for (int64_t b = 0; b < nb; ++b) {
    const int l = P->level[b];
    const double sd = P->W / (double)(1ll << l);
    for (int d = 0; d < 3; ++d) geom[4 * b + d] = (T)((P->anchor[3 * b + d] + 0.5) * sd - 0.5 * P->W);
    geom[4 * b + 3] = (T)(0.5 * sd);
  }
  if ((rc = upload(P, &P->dt.box_geom, geom))) return rc;
  return FMM_OK;
}

// ---------------------------------------------------------------------------
// Device lists
// ---------------------------------------------------------------------------
static int upload_lists(fmm_plan *P) {
  const int64_t nb = (int64_t)P->level.size();
  DevTree &D = P->dt;
  D.nbox = (int)nb;
  D.maxlevel = (int)P->level_begin.size() - 2;
  std::vector<int32_t> bb(nb), be(nb);
  for (int64_t b = 0; b < nb; ++b) { bb[b] = (int32_t)P->begin[b]; be[b] = (int32_t)P->end[b]; }
  int rc;
  if ((rc = upload(P, (void **)&D.box_begin, bb))) return rc;
  if ((rc = upload(P, (void **)&D.box_end, be))) return rc;
  // Leaf work.  Near sources are point ranges: the U list, W-list boxes
  // holding at most n_surf points (their points are cheaper and exact
  // compared with their equivalent surface) and, for leaves with at most
  // n_surf targets, the X list (evaluated at the targets instead of on the
  // leaf's check surface).  Far sources are surfaces: the remaining W-list
  // boxes (upward equivalent) and the leaf's own downward equivalent surface.
  const int64_t ns = P->nsurf;
  std::vector<int32_t> leaves, hl, p2m, p2mo = {0};
  std::vector<char> x_direct(nb, 0);
  int64_t inter = 0, far_inter = 0;
  // Points are stored relative to their leaf's centre, so every near range
  // holds the points of one leaf and carries that leaf (its centre offset
  // from the target leaf is applied once per range).  Leaves by first point,
  // to cut the range of a non-leaf W-list box into its leaves.
  std::vector<std::pair<int64_t, int64_t>> leaf_at;  // (first point, box)
  for (int64_t b = 0; b < nb; ++b)
    if (!P->nchild[b] && P->end[b] > P->begin[b]) leaf_at.push_back({P->begin[b], b});
  std::sort(leaf_at.begin(), leaf_at.end());
  // per leaf slot: near ranges (one source leaf each) and far surface boxes
  // (bit 30 marks the leaf's own downward surface)
  struct Rng { int32_t j0, j1, src; };
  struct LeafSrc { std::vector<Rng> near; std::vector<int32_t> far; int64_t m; };
  std::vector<LeafSrc> src;
  for (int64_t b = 0; b < nb; ++b) {
    if (P->nchild[b]) continue;
    leaves.push_back((int32_t)b);
    LeafSrc L;
    L.m = P->end[b] - P->begin[b];
    std::vector<Rng> rg;
    auto add_range = [&](int64_t a) {
      if (!P->nchild[a]) {  // a leaf is its own range
        if (P->end[a] > P->begin[a]) rg.push_back({(int32_t)P->begin[a], (int32_t)P->end[a], (int32_t)a});
        inter += L.m * (P->end[a] - P->begin[a]);
        return;
      }
      auto it = std::lower_bound(leaf_at.begin(), leaf_at.end(), std::make_pair(P->begin[a], (int64_t)-1));
      for (; it != leaf_at.end() && it->first < P->end[a]; ++it) {
        const int64_t lf = it->second;
        rg.push_back({(int32_t)P->begin[lf], (int32_t)P->end[lf], (int32_t)lf});
      }
      inter += L.m * (P->end[a] - P->begin[a]);
    };
    for (int64_t k = P->loff[0][b]; k < P->loff[0][b + 1]; ++k) add_range(P->lidx[0][k]);
    for (int64_t k = P->loff[2][b]; k < P->loff[2][b + 1]; ++k) {
      const int64_t a = P->lidx[2][k];
      if (P->end[a] - P->begin[a] <= ns) add_range(a);
      else L.far.push_back((int32_t)a);
    }
    if (L.m <= ns) {
      x_direct[b] = 1;
      for (int64_t k = P->loff[3][b]; k < P->loff[3][b + 1]; ++k) add_range(P->lidx[3][k]);
    }
    if (P->level[b] >= 2) L.far.push_back((int32_t)b | (1 << 30));
    // in point order (disjoint ranges)
    std::sort(rg.begin(), rg.end(), [](const Rng &x, const Rng &y) { return x.j0 < y.j0; });
    L.near = std::move(rg);
    far_inter += L.m * ns * (int64_t)L.far.size();
    hl.push_back(P->level[b] >= 2 ? 1 : 0);
    if (P->level[b] >= 2) { p2m.push_back((int32_t)b); p2mo.push_back((int32_t)p2m.size()); }
    src.push_back(std::move(L));
  }
  // Tiles of 64 targets (a tile of at most 32 or 16 targets runs split: 2 or
  // 4 sub-waves take the same targets and the sources in turn).  A tile whose
  // source work exceeds `cap` is cut into parts of about `cap` (near ranges
  // cut at point boundaries, surfaces whole); parts write partial sums that
  // k_leaf_parts adds in part order.  With the waves of one launch resident
  // at once, capping the work per wave is what balances the SIMDs.
  const double far_w = P->tune.far_weight;  // a surface source also computes its position
  struct Tile { double cost; int32_t slot, t0, split; };
  std::vector<Tile> tiles;
  double total = 0;
  for (size_t sl = 0; sl < src.size(); ++sl) {
    double c = 0;
    for (auto &r : src[sl].near) c += r.j1 - r.j0;
    c += far_w * ns * (double)src[sl].far.size();
    for (int64_t t0 = 0; t0 < src[sl].m; t0 += 64) {
      const int64_t rem = src[sl].m - t0;
      const int split = rem <= P->tune.tile_split4 ? 4 : (rem <= P->tune.tile_split2 ? 2 : 1);
      tiles.push_back({c / split, (int32_t)sl, (int32_t)t0, split});
      total += c / split;
    }
  }
  const double cap = std::max((double)P->tune.work_cap_min, total / (double)P->tune.work_cap_div);
  // an item of a whole tile reads its leaf's range lists (whole = true);
  // the parts of a split tile carry their own cut lists
  struct Item { double cost; int32_t slot, code, part; bool whole; std::vector<Rng> near; std::vector<int32_t> far; };
  std::vector<Item> items;
  std::vector<int32_t> split_tiles;  // (slot, code, first part, nparts)
  int32_t nparts_total = 0;
  for (const Tile &t : tiles) {
    const LeafSrc &L = src[t.slot];
    const int32_t code = t.t0 | (t.split << 24);
    const int nparts = (int)std::ceil(t.cost / cap - 1e-9);
    if (nparts <= 1) {
      items.push_back({t.cost, t.slot, code, -1, true, {}, {}});
      continue;
    }
    const double per = t.cost * t.split / nparts;  // unsplit-source units per part
    split_tiles.push_back(t.slot); split_tiles.push_back(code);
    split_tiles.push_back(nparts_total);
    int made = 0;
    Item cur{0, t.slot, code, nparts_total, false, {}, {}};
    double acc = 0;
    auto flush = [&]() {
      cur.cost = acc / t.split;
      cur.part = nparts_total++;
      items.push_back(std::move(cur));
      ++made;
      cur = Item{0, t.slot, code, 0, false, {}, {}};
      acc = 0;
    };
    for (auto r : L.near) {
      int32_t j = r.j0;
      while (j < r.j1) {
        const int32_t take = (int32_t)std::max<double>(1.0, std::min<double>(r.j1 - j, per - acc));
        cur.near.push_back({j, j + take, r.src});
        acc += take;
        j += take;
        if (acc >= per - 0.5 && made < nparts - 1) flush();
      }
    }
    for (int32_t f : L.far) {
      cur.far.push_back(f);
      acc += far_w * ns;
      if (acc >= per - 0.5 && made < nparts - 1) flush();
    }
    if (!cur.near.empty() || !cur.far.empty() || made == 0) flush();
    split_tiles.push_back(made);
  }
  // longest items first (a stable sort of their indices)
  std::vector<int32_t> order(items.size());
  for (size_t i = 0; i < items.size(); ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return items[x].cost > items[y].cost; });
  // centre of box b relative to its molecule's root centre (FP64)
  auto cen = [&](int64_t b, int d) {
    const double sd = P->W / (double)(1ll << P->level[b]);
    return (P->anchor[3 * b + d] + 0.5) * sd - 0.5 * P->W;
  };
  // near_o: per range, the source leaf's centre minus the target leaf's;
  // far_o: per far entry, the surface box centre minus the target leaf's and
  // the surface radius
  std::vector<int32_t> it4, no = {0}, nrng, fo = {0}, far;
  std::vector<double> near_o, far_o;
  P->item_pairs.clear();
  for (const int32_t io : order) {
    const Item &it = items[io];
    const int64_t tb = leaves[it.slot];
    const std::vector<Rng> &inear = it.whole ? src[it.slot].near : it.near;
    const std::vector<int32_t> &ifar = it.whole ? src[it.slot].far : it.far;
    it4.push_back(it.slot); it4.push_back(it.code); it4.push_back(it.part); it4.push_back(0);
    int64_t nsrc = 0;
    for (auto &r : inear) nsrc += r.j1 - r.j0;
    P->item_pairs.push_back(std::min<int64_t>(64, src[it.slot].m - (it.code & 0xffffff)) * nsrc);
    for (auto &r : inear) {
      nrng.push_back(r.j0); nrng.push_back(r.j1);
      for (int d = 0; d < 3; ++d) near_o.push_back(cen(r.src, d) - cen(tb, d));
      near_o.push_back(0.0);
    }
    no.push_back((int32_t)(nrng.size() / 2));
    for (int32_t f : ifar) {
      const bool own = (f >> 30) & 1;
      const int64_t a = f & 0x3fffffff;
      const double h = 0.5 * P->W / (double)(1ll << P->level[a]);
      for (int d = 0; d < 3; ++d) far_o.push_back(cen(a, d) - cen(tb, d));
      far_o.push_back(h * (own ? ALPHA_DE : ALPHA_UE));
    }
    far.insert(far.end(), ifar.begin(), ifar.end());
    fo.push_back((int32_t)far.size());
  }
  P->leaf_ids = leaves;
  P->p2p_inter = inter;
  P->far_inter = far_inter;
  D.nleaf = (int)leaves.size();
  D.nitems = (int)items.size();
  D.nsplit = (int)(split_tiles.size() / 4);
  D.nparts = nparts_total;
  if ((rc = upload(P, (void **)&D.leaves, leaves))) return rc;
  if ((rc = upload(P, (void **)&D.items, it4))) return rc;
  if ((rc = upload(P, (void **)&D.near_off, no))) return rc;
  if ((rc = upload(P, (void **)&D.near_rng, nrng))) return rc;
  if ((rc = upload_real(P, &D.near_o, near_o))) return rc;
  if ((rc = upload_real(P, &D.far_o, far_o))) return rc;
  if ((rc = upload(P, (void **)&D.far_off, fo))) return rc;
  if ((rc = upload(P, (void **)&D.far_idx, far))) return rc;
  if ((rc = upload(P, (void **)&D.split_tiles, split_tiles))) return rc;
  if ((rc = upload(P, (void **)&P->d_has_local, hl))) return rc;
  P->p2m_count = (int)p2m.size();
  if ((rc = upload(P, (void **)&P->d_p2m_box, p2m))) return rc;
  if ((rc = upload(P, (void **)&P->d_p2m_off, p2mo))) return rc;
  // P2L: X lists of the boxes whose X list is not evaluated directly
  std::vector<int32_t> xb, xo = {0}, xi;
  std::vector<double> x_o;  // per X entry: source leaf centre minus target box centre
  for (int64_t b = 0; b < nb; ++b) {
    if (P->loff[3][b + 1] == P->loff[3][b] || x_direct[b]) continue;
    xb.push_back((int32_t)b);
    for (int64_t k = P->loff[3][b]; k < P->loff[3][b + 1]; ++k) {
      const int64_t a = P->lidx[3][k];  // a leaf
      xi.push_back((int32_t)a);
      for (int d = 0; d < 3; ++d) x_o.push_back(cen(a, d) - cen(b, d));
      x_o.push_back(0.0);
    }
    xo.push_back((int32_t)xi.size());
  }
  D.nxbox = (int)xb.size();
  P->p2l_boxes = xb;
  if ((rc = upload(P, (void **)&D.x_box, xb))) return rc;
  if ((rc = upload(P, (void **)&D.x_off, xo))) return rc;
  if ((rc = upload(P, (void **)&D.x_idx, xi))) return rc;
  if ((rc = upload_real(P, &D.x_o, x_o))) return rc;
  // V pairs in GEMM order, (level, offset code, target): a counting sort over
  // the 343 offset codes of each level, stable in target order (boxes and
  // their V lists are visited in order).  vpp gives, per V-list entry in
  // target-major order (the order of each box's sum: its V list, ascending
  // source id), the pair's position in GEMM order.
  {
    const int64_t nv = P->loff[1][nb];
    const int nbucket = (MAXLEVEL + 1) * 343;
    std::vector<int32_t> bucket((size_t)nv);
    std::vector<int64_t> cursor((size_t)nbucket + 1, 0);
    for (int64_t b = 0; b < nb; ++b)
      for (int64_t k = P->loff[1][b]; k < P->loff[1][b + 1]; ++k) {
        const int64_t a = P->lidx[1][k];
        const int c = m2l_code((int)(P->anchor[3 * a] - P->anchor[3 * b]),
                               (int)(P->anchor[3 * a + 1] - P->anchor[3 * b + 1]),
                               (int)(P->anchor[3 * a + 2] - P->anchor[3 * b + 2]));
        bucket[k] = P->level[b] * 343 + c;
        cursor[bucket[k] + 1]++;
      }
    for (int i = 0; i < nbucket; ++i) cursor[i + 1] += cursor[i];
    P->vpair_src.resize((size_t)nv);
    P->vpair_tgt.resize((size_t)nv);
    std::vector<int32_t> vpp((size_t)nv);
    for (int64_t b = 0; b < nb; ++b)
      for (int64_t k = P->loff[1][b]; k < P->loff[1][b + 1]; ++k) {
        const int64_t pos = cursor[bucket[k]]++;
        P->vpair_src[pos] = (int32_t)P->lidx[1][k];
        P->vpair_tgt[pos] = (int32_t)b;
        vpp[k] = (int32_t)pos;
      }
    // every box at level >= 2 gets its sum (possibly empty); those boxes
    // are the last ones (boxes are ordered by level) and hold every V entry
    std::vector<int32_t> vt, vo;
    const int64_t b2 = P->level_begin.size() > 2 ? P->level_begin[2] : nb;
    for (int64_t b = b2; b < nb; ++b) {
      vt.push_back((int32_t)b);
      vo.push_back((int32_t)(P->loff[1][b] - P->loff[1][b2]));
    }
    vo.push_back((int32_t)(P->loff[1][nb] - P->loff[1][b2]));
    if (P->loff[1][b2] != 0) {
      set_error("internal: V lists above level 2");
      return FMM_EINVAL;
    }
    D.nvbox = (int)vt.size();
    D.nvpair = nv;
    if ((rc = upload(P, (void **)&D.v_tgt, vt))) return rc;
    if ((rc = upload(P, (void **)&D.v_off, vo))) return rc;
    if ((rc = upload(P, (void **)&D.v_pair, vpp))) return rc;
  }
  // M2M sums: per level, the non-leaf boxes and their children (octant order)
  D.m2m_tgt.assign(D.maxlevel + 1, nullptr);
  D.m2m_off.assign(D.maxlevel + 1, nullptr);
  D.m2m_kid.assign(D.maxlevel + 1, nullptr);
  D.m2m_n.assign(D.maxlevel + 1, 0);
  for (int l = 2; l < D.maxlevel; ++l) {
    std::vector<int32_t> tg, of = {0}, kd;
    for (int64_t b = P->level_begin[l]; b < P->level_begin[l + 1]; ++b) {
      if (!P->nchild[b]) continue;
      tg.push_back((int32_t)b);
      for (int k = 0; k < P->nchild[b]; ++k) kd.push_back((int32_t)(P->child_begin[b] + k));
      of.push_back((int32_t)kd.size());
    }
    D.m2m_n[l] = (int)tg.size();
    if ((rc = upload(P, (void **)&D.m2m_tgt[l], tg))) return rc;
    if ((rc = upload(P, (void **)&D.m2m_off[l], of))) return rc;
    if ((rc = upload(P, (void **)&D.m2m_kid[l], kd))) return rc;
  }
  return FMM_OK;
}

static void add_columns(GemmBatch &bt, int mat, double alpha, const std::vector<int32_t> &src,
                        const std::vector<int32_t> &dst) {
  // src has S entries per column; split into tasks of bt.nt columns
  const int nc = (int)dst.size();
  const int base = (int)bt.h_dst.size();
  for (int c0 = 0; c0 < nc; c0 += bt.nt) {
    GemmTask t;
    t.mat = mat;
    t.col0 = base + c0;
    t.ncol = std::min(bt.nt, nc - c0);
    t.nrb = 0;
    t.klen = 0;
    t.alpha = alpha;
    bt.h_tasks.push_back(t);
  }
  bt.h_src.insert(bt.h_src.end(), src.begin(), src.end());
  bt.h_dst.insert(bt.h_dst.end(), dst.begin(), dst.end());
}

static int finish_batch(fmm_plan *P, GemmBatch &bt) {
  const int64_t nmat = bt.pool == 0 ? P->pool1_count : P->poolbf_count;
  for (const GemmTask &t : bt.h_tasks)
    if (t.mat < 0 || t.mat >= nmat) {
      set_error("internal: GEMM task references a missing operator");
      return FMM_EINVAL;
    }
  bt.ntask = (int)bt.h_tasks.size();
  bt.ncols = (int)bt.h_dst.size();
  int rc;
  if ((rc = upload(P, (void **)&bt.d_tasks, bt.h_tasks))) return rc;
  if ((rc = upload(P, (void **)&bt.d_src, bt.h_src))) return rc;
  if ((rc = upload(P, (void **)&bt.d_dst, bt.h_dst))) return rc;
  bt.h_tasks.clear(); bt.h_tasks.shrink_to_fit();
  bt.h_src.clear(); bt.h_src.shrink_to_fit();
  bt.h_dst.clear(); bt.h_dst.shrink_to_fit();
  return FMM_OK;
}

// Row length of the M2L pair slots: the largest downward rank, rounded up to
// 16 (the rows the M2L GEMM computes).
static int pair_ld(const fmm_plan *P) {
  int m = 16;
  for (int l = 2; l <= P->dt.maxlevel; ++l) m = std::max(m, std::max(16, ((P->rank_d[l] + 15) / 16) * 16));
  return m;
}

int ensure_lists(fmm_plan *P, int nr) {
  PassLists &L = P->lists_by_nr[nr];
  if (L.nr == nr) return FMM_OK;
  const int maxl = P->dt.maxlevel;
  const int ld = P->ld;
  const int64_t nb = (int64_t)P->level.size();
  const int64_t ns = P->nsurf;
  int rc;
  std::vector<int32_t> src, dst;
  auto cols_for = [&](const std::vector<int64_t> &boxes_src, const std::vector<int64_t> &boxes_dst) {
    src.clear(); dst.clear();
    for (size_t i = 0; i < boxes_dst.size(); ++i)
      for (int r = 0; r < nr; ++r) {
        src.push_back((int32_t)(boxes_src[i] * nr + r));
        dst.push_back((int32_t)(boxes_dst[i] * nr + r));
      }
  };
  auto r16 = [](int r) { return std::max(16, ((r + 15) / 16) * 16); };
  auto oct_of = [&](int64_t b) {
    return (int)(((P->anchor[3 * b] & 1) << 2) | ((P->anchor[3 * b + 1] & 1) << 1) | (P->anchor[3 * b + 2] & 1));
  };
  int maxru = 16, maxrd = 16;
  for (int l = 2; l <= maxl; ++l) { maxru = std::max(maxru, r16(P->rank_u[l])); maxrd = std::max(maxrd, r16(P->rank_d[l])); }
  const int L1 = std::max(maxl + 1, 0);
  L.m2m.assign(L1, GemmBatch()); L.l2l.assign(L1, GemmBatch());
  L.ut_u_all = GemmBatch(); L.vs_u = GemmBatch(); L.ut_dx = GemmBatch(); L.vs_d = GemmBatch(); L.m2l = GemmBatch();
  L.ut_u_all.nrb = maxru / 16; L.ut_u_all.klen = ld;
  L.vs_u.nrb = ld / 16; L.vs_u.klen = maxru;
  L.ut_dx.nrb = maxrd / 16; L.ut_dx.klen = ld;
  L.vs_d.nrb = ld / 16; L.vs_d.klen = maxrd;
  L.m2l.nrb = maxrd / 16; L.m2l.klen = maxru; L.m2l.ldy = pair_ld(P);
  if (P->precision == FMM_FP32_BF16X3) {
    L.m2l.pool = 2;
    L.m2l.klen = std::min(((maxru + 31) / 32) * 32, P->bf_kb * 32);
    if (P->tune.m2l_cols == 2 * GEMM_NT && !P->tune.m2l_factored) L.m2l.nt = 2 * GEMM_NT;
  }
  // factored M2L: R maps upward coordinates (k <= maxru) to intermediates of
  // m2l_ldt values per pair; L reads those rows
  const bool fact = P->tune.m2l_factored != 0;
  L.m2l_r = GemmBatch();
  if (fact) {
    L.m2l_r.pool = L.m2l.pool;
    L.m2l_r.klen = L.m2l.klen;
    L.m2l_r.nrb = P->m2l_ldt / 16;
    L.m2l_r.ldy = P->m2l_ldt;
    L.m2l.ldx = P->m2l_ldt;
    L.m2l.klen = P->m2l_ldt;
  }
  // boxes whose upward equivalent density is evaluated (M2P sources)
  std::vector<char> need_equ(nb, 0);
  for (int64_t b = 0; b < nb; ++b) {
    if (P->nchild[b]) continue;
    for (int64_t k = P->loff[2][b]; k < P->loff[2][b + 1]; ++k) {
      const int64_t a = P->lidx[2][k];
      if (P->end[a] - P->begin[a] > ns) need_equ[a] = 1;
    }
  }
  for (int l = 2; l <= maxl; ++l) {
    std::vector<int64_t> leaves, all;
    for (int64_t b = P->level_begin[l]; b < P->level_begin[l + 1]; ++b) {
      all.push_back(b);
      if (!P->nchild[b]) leaves.push_back(b);
    }
    // upward: M2M slots, one per child box at level l + 1 (grouped by
    // octant), summed per parent by k_pair_reduce
    if (l < maxl) {
      GemmBatch &bt = L.m2m[l];
      bt.nrb = r16(P->rank_u[l]) / 16;
      bt.klen = r16(P->rank_u[l + 1]);
      for (int oct = 0; oct < 8; ++oct) {
        std::vector<int64_t> kids;
        for (int64_t b = P->level_begin[l + 1]; b < P->level_begin[l + 2]; ++b)
          if (oct_of(b) == oct) kids.push_back(b);
        if (kids.empty()) continue;
        cols_for(kids, kids);
        add_columns(bt, P->m2m_id[l][oct], 1.0, src, dst);
      }
      if ((rc = finish_batch(P, bt))) return rc;
    }
    // upward: leaves' check potentials to singular coordinates (one batch
    // for every level, launched before the M2M sweep)
    cols_for(leaves, leaves);
    if (!dst.empty()) add_columns(L.ut_u_all, P->utu_id[l], 1.0, src, dst);
    // upward equivalent densities of the M2P sources
    std::vector<int64_t> eb;
    for (int64_t b : all) if (need_equ[b]) eb.push_back(b);
    cols_for(eb, eb);
    if (!dst.empty()) add_columns(L.vs_u, P->vsu_id[l], P->vs_alpha[l], src, dst);
    // downward: L2L between singular coordinates (levels >= 3)
    if (l >= 3) {
      GemmBatch &bt = L.l2l[l];
      bt.mode = GEMM_ADD;
      bt.nrb = r16(P->rank_d[l]) / 16;
      bt.klen = r16(P->rank_d[l - 1]);
      for (int oct = 0; oct < 8; ++oct) {
        std::vector<int64_t> bs, bd;
        for (int64_t b : all) {
          if (oct_of(b) != oct) continue;
          bs.push_back(P->parent[b]);
          bd.push_back(b);
        }
        if (bd.empty()) continue;
        cols_for(bs, bd);
        add_columns(bt, P->l2l_id[l - 1][oct], 1.0, src, dst);
      }
      if ((rc = finish_batch(P, bt))) return rc;
    }
    // downward equivalent densities of the leaves
    cols_for(leaves, leaves);
    if (!dst.empty()) add_columns(L.vs_d, P->vsd_id[l], P->vs_alpha[l], src, dst);
  }
  // P2L boxes: their check potentials to singular coordinates (added)
  {
    std::vector<int64_t> xb;
    for (int32_t b : P->p2l_boxes) xb.push_back(b);
    std::stable_sort(xb.begin(), xb.end(), [&](int64_t x, int64_t y) { return P->level[x] < P->level[y]; });
    size_t i = 0;
    while (i < xb.size()) {
      size_t j = i;
      while (j < xb.size() && P->level[xb[j]] == P->level[xb[i]]) ++j;
      std::vector<int64_t> part(xb.begin() + i, xb.begin() + j);
      cols_for(part, part);
      add_columns(L.ut_dx, P->utd_id[P->level[xb[i]]], 1.0, src, dst);
      i = j;
    }
  }
  if ((rc = finish_batch(P, L.ut_u_all))) return rc;
  if ((rc = finish_batch(P, L.vs_u))) return rc;
  if ((rc = finish_batch(P, L.ut_dx))) return rc;
  if ((rc = finish_batch(P, L.vs_d))) return rc;
  // M2L: pairs in GEMM order, tasks split at (level, offset) changes
  {
    const int64_t np = (int64_t)P->vpair_src.size();
    auto code_of = [&](int64_t j) {
      const int64_t t = P->vpair_tgt[j], a = P->vpair_src[j];
      return m2l_code((int)(P->anchor[3 * a] - P->anchor[3 * t]), (int)(P->anchor[3 * a + 1] - P->anchor[3 * t + 1]),
                      (int)(P->anchor[3 * a + 2] - P->anchor[3 * t + 2]));
    };
    int64_t i = 0;
    L.m2l_t0.assign((size_t)maxl + 2, -1);
    while (i < np) {
      const int l = P->level[P->vpair_tgt[i]];
      const int code = code_of(i);
      if (L.m2l_t0[l] < 0) L.m2l_t0[l] = (int)L.m2l.h_tasks.size();
      int64_t j = i;
      src.clear(); dst.clear();
      while (j < np && P->level[P->vpair_tgt[j]] == l && code_of(j) == code) {
        for (int r = 0; r < nr; ++r) {
          src.push_back((int32_t)(P->vpair_src[j] * nr + r));
          dst.push_back((int32_t)(j * nr + r));
        }
        ++j;
      }
      // only the rows of this level's downward rank and the columns of its
      // upward rank (the rest of the operator is zero padding; the bf16x3
      // kernel steps k by 32)
      auto kround = [&](int r) { return L.m2l.pool == 2 ? ((r16(r) + 31) / 32) * 32 : r16(r); };
      if (fact) {
        // R: upward coordinates -> the pair's k-value intermediate (row j);
        // L: intermediate -> the pair's slot
        const int kf = P->m2l_k[l][code];
        std::vector<int32_t> mid(dst);
        size_t t0 = L.m2l_r.h_tasks.size();
        add_columns(L.m2l_r, P->m2l_r_id[l][code], 1.0, src, mid);
        for (size_t t = t0; t < L.m2l_r.h_tasks.size(); ++t) {
          L.m2l_r.h_tasks[t].nrb = r16(kf) / 16;
          L.m2l_r.h_tasks[t].klen = kround(P->rank_u[l]);
        }
        t0 = L.m2l.h_tasks.size();
        add_columns(L.m2l, P->m2l_id[l][code], 1.0, mid, dst);
        for (size_t t = t0; t < L.m2l.h_tasks.size(); ++t) {
          L.m2l.h_tasks[t].nrb = r16(P->rank_d[l]) / 16;
          L.m2l.h_tasks[t].klen = kround(kf);
        }
      } else {
        const size_t t0 = L.m2l.h_tasks.size();
        add_columns(L.m2l, P->m2l_id[l][code], 1.0, src, dst);
        for (size_t t = t0; t < L.m2l.h_tasks.size(); ++t) {
          L.m2l.h_tasks[t].nrb = r16(P->rank_d[l]) / 16;
          L.m2l.h_tasks[t].klen = kround(P->rank_u[l]);
        }
      }
      i = j;
    }
  }
  if (L.m2l_t0.size() != (size_t)maxl + 2) L.m2l_t0.assign((size_t)maxl + 2, -1);
  L.m2l_t0[maxl + 1] = (int)L.m2l.h_tasks.size();
  for (int l = maxl; l >= 0; --l)
    if (L.m2l_t0[l] < 0) L.m2l_t0[l] = L.m2l_t0[l + 1];
  if ((rc = finish_batch(P, L.m2l))) return rc;
  if (fact && (rc = finish_batch(P, L.m2l_r))) return rc;
  if (!P->d_m2l_rows) {
    std::vector<int32_t> rows(std::max<int64_t>(1, nb), 16);
    for (int64_t b = 0; b < nb; ++b)
      if (P->level[b] >= 2) rows[b] = r16(P->rank_d[P->level[b]]);
    if ((rc = upload(P, (void **)&P->d_m2l_rows, rows))) return rc;
  }
  L.nr = nr;
  return FMM_OK;
}

// FNV-1a over everything the shared launches of a pair evaluation depend on:
// the input coordinates (their checksum from the bounding-box pass), the root
// cube side and the molecules' corners, point order, molecule ranges, boxes,
// surface size and the item lists.  Two plans with equal fingerprints share
// one tree: the same sorted points, box geometry, near ranges and items.
static uint64_t tree_fingerprint(const fmm_plan *P) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void *data, size_t bytes) {
    const unsigned char *c = (const unsigned char *)data;
    for (size_t i = 0; i < bytes; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  };
  mix(&P->coord_hash, sizeof(P->coord_hash));
  mix(&P->W, sizeof(P->W));
  mix(P->mol_lo.data(), P->mol_lo.size() * sizeof(double));
  mix(&P->n, sizeof(P->n));
  mix(&P->nsurf, sizeof(P->nsurf));
  mix(&P->ncrit, sizeof(P->ncrit));
  mix(P->perm.data(), P->perm.size() * sizeof(int64_t));
  mix(P->mol_off.data(), P->mol_off.size() * sizeof(int64_t));
  mix(P->begin.data(), P->begin.size() * sizeof(int64_t));
  mix(P->end.data(), P->end.size() * sizeof(int64_t));
  mix(P->anchor.data(), P->anchor.size() * sizeof(int64_t));
  mix(&P->dt.nitems, sizeof(P->dt.nitems));
  mix(&P->dt.nparts, sizeof(P->dt.nparts));
  mix(&P->dt.nsplit, sizeof(P->dt.nsplit));
  return h;
}

// Side streams of pair evaluations: three per device for the whole process
// (default priority, created on first use, kept until the process ends).
// Every plan pair on a device queues its far-field passes, its early
// near-field items and its early M2L levels on the same three streams, so the hardware queues the
// library takes do not grow with the number of live plans.  HIP spreads
// streams over a small pool of hardware queues (four by default); with
// streams of their own, the plans set up after enough others had theirs land
// on the caller's queue, and their side passes then wait behind the near
// field instead of running beside it.
static std::mutex g_side_mu;
static std::map<int, std::array<hipStream_t, 3>> g_side;

static int side_streams(int device, hipStream_t *aux, hipStream_t *aux2, hipStream_t *aux3) {
  std::lock_guard<std::mutex> lock(g_side_mu);
  auto it = g_side.find(device);
  if (it == g_side.end()) {
    int cur = 0;
    FMM_HIP_TRY(hipGetDevice(&cur));
    if (cur != device) FMM_HIP_TRY(hipSetDevice(device));
    std::array<hipStream_t, 3> st{nullptr, nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (hipStream_t &x : st)
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) {
      for (hipStream_t x : st)
        if (x) (void)hipStreamDestroy(x);
      FMM_HIP_TRY(e);
    }
    it = g_side.emplace(device, st).first;
  }
  *aux = it->second[0];
  *aux2 = it->second[1];
  *aux3 = it->second[2];
  return FMM_OK;
}

// Resources of a pair evaluation (A: Laplace half, B: Yukawa half): the
// device's side streams that run both kernels' passes, A's fork and join
// events and its event marking the end of the upward pass, B's events marking
// the end of the surface passes and of the P2L projections, and A's buffer of
// near-field running sums for nr columns.
int ensure_pair(fmm_plan *A, fmm_plan *B, int nr) {
  if (!A->aux || !A->aux2 || !A->aux3) {
    int rc;
    if ((rc = side_streams(A->device, &A->aux, &A->aux2, &A->aux3))) return rc;
  }
  if (!A->ev_near) FMM_HIP_TRY(hipEventCreateWithFlags(&A->ev_near, hipEventDisableTiming));
  if (!A->ev_fork) FMM_HIP_TRY(hipEventCreateWithFlags(&A->ev_fork, hipEventDisableTiming));
  if (!A->ev_join) FMM_HIP_TRY(hipEventCreateWithFlags(&A->ev_join, hipEventDisableTiming));
  if (!A->ev_up) FMM_HIP_TRY(hipEventCreateWithFlags(&A->ev_up, hipEventDisableTiming));
  if (!A->ev_m2l) FMM_HIP_TRY(hipEventCreateWithFlags(&A->ev_m2l, hipEventDisableTiming));
  if (!A->ev_m2m) FMM_HIP_TRY(hipEventCreateWithFlags(&A->ev_m2m, hipEventDisableTiming));
  if (!A->ev_m2lf) FMM_HIP_TRY(hipEventCreateWithFlags(&A->ev_m2lf, hipEventDisableTiming));
  if (!B->ev_fork) FMM_HIP_TRY(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
  if (!B->ev_join) FMM_HIP_TRY(hipEventCreateWithFlags(&B->ev_join, hipEventDisableTiming));
  const size_t es = A->precision == FMM_FP64 ? 8 : 4;
  const size_t need = std::max<size_t>(1, (size_t)A->dt.nitems) * 2 * nr * 4 * 64 * es;
  if (A->pair_acc_bytes < need) {
    int rc;
    if ((rc = dev_alloc(A, &A->pair_acc, need))) return rc;
    A->pair_acc_bytes = need;
  }
  return FMM_OK;
}

int ensure_pair_md(fmm_plan *A, fmm_plan *B) {
  (void)B;
  if (A->dips) return FMM_OK;
  const size_t es = A->precision == FMM_FP64 ? 8 : 4;
  return dev_alloc(A, &A->dips, std::max<size_t>(1, (size_t)A->n) * 4 * es);
}

int ensure_work(fmm_plan *P, int nr) {
  if (P->work_nr >= nr) return FMM_OK;
  const size_t es = P->precision == FMM_FP64 ? 8 : 4;
  const int64_t nb = P->dt.nbox;
  const size_t wbytes = (size_t)nb * nr * P->ld * es;
  int rc;
  // old buffers stay in allocs until fmm_free (simple and safe for in-flight work)
  if ((rc = dev_alloc(P, &P->qs, (size_t)P->n * nr * es))) return rc;
  if ((rc = dev_alloc(P, &P->equ, wbytes))) return rc;
  if ((rc = dev_alloc(P, &P->chk, wbytes))) return rc;
  if ((rc = dev_alloc(P, &P->eqd, wbytes))) return rc;
  if ((rc = dev_alloc(P, &P->chku, wbytes))) return rc;
  if ((rc = dev_alloc(P, &P->cu, wbytes))) return rc;
  if ((rc = dev_alloc(P, &P->yd, wbytes))) return rc;
  if ((rc = dev_alloc(P, &P->mslot, wbytes))) return rc;
  if ((rc = dev_alloc(P, &P->ydx, wbytes))) return rc;
  if ((rc = dev_alloc(P, &P->pairbuf, (size_t)std::max<int64_t>(1, P->dt.nvpair) * nr * pair_ld(P) * es))) return rc;
  if (P->m2l_ldt > 0 &&
      (rc = dev_alloc(P, &P->m2l_t, (size_t)std::max<int64_t>(1, P->dt.nvpair) * nr * P->m2l_ldt * es)))
    return rc;
  // padding rows/columns must hold zeros (the GEMM K dimension reads them)
  FMM_HIP_TRY(hipMemset(P->equ, 0, wbytes));
  FMM_HIP_TRY(hipMemset(P->chk, 0, wbytes));
  FMM_HIP_TRY(hipMemset(P->eqd, 0, wbytes));
  FMM_HIP_TRY(hipMemset(P->chku, 0, wbytes));
  FMM_HIP_TRY(hipMemset(P->cu, 0, wbytes));
  FMM_HIP_TRY(hipMemset(P->yd, 0, wbytes));
  // rows of boxes without an X list stay zero: the M2L sums add this array
  FMM_HIP_TRY(hipMemset(P->ydx, 0, wbytes));
  P->work_nr = nr;
  return FMM_OK;
}

hipEvent_t prof_begin(fmm_plan *P, int phase, hipStream_t s) {
  if (!((P->profiling >> phase) & 1)) return nullptr;
  hipEvent_t e = nullptr;
  if (!P->event_pool.empty()) {
    e = P->event_pool.back();
    P->event_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return nullptr;
  }
  (void)hipEventRecord(e, s);
  return e;
}

void prof_launch(fmm_plan *P, int phase, hipEvent_t *begin, hipEvent_t *end) {
  *begin = *end = nullptr;
  if (!((P->profiling >> phase) & 1)) return;
  hipEvent_t ev[2] = {nullptr, nullptr};
  for (hipEvent_t &e : ev) {
    if (!P->event_pool.empty()) {
      e = P->event_pool.back();
      P->event_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
      if (ev[0]) P->event_pool.push_back(ev[0]);
      return;
    }
  }
  P->prof_events.push_back({phase, {ev[0], ev[1]}});
  *begin = ev[0];
  *end = ev[1];
}

void prof_end(fmm_plan *P, int phase, hipEvent_t begin, hipStream_t s) {
  if (!P->profiling || !begin) return;
  hipEvent_t e = nullptr;
  if (!P->event_pool.empty()) {
    e = P->event_pool.back();
    P->event_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    return;
  }
  (void)hipEventRecord(e, s);
  P->prof_events.push_back({phase, {begin, e}});
}

// Tunables for plans set up from now on (fmm_set_tuning).
static std::mutex g_tune_mu;
static fmm_tuning_t g_tune{32, 16, 512, 16384, 1.15, 0, 0, 4, 0, 512, 0, 64, 0, 0, 1024, 0, 0};

// Live plans whose tree later plans on the same points may share.
static std::mutex g_tree_mu;
static std::vector<fmm_plan *> g_tree_plans;

// A live plan whose tree P can take: the same input coordinates (checksum
// over their bits, point count and molecule ranges), root cube, ncrit,
// surface size (the leaf items depend on it), working type and device.
static fmm_plan *find_tree(const fmm_plan *P) {
  std::lock_guard<std::mutex> lock(g_tree_mu);
  for (fmm_plan *A : g_tree_plans)
    if (A->coord_hash == P->coord_hash && A->n == P->n && A->mol_off == P->mol_off && A->W == P->W &&
        A->mol_lo == P->mol_lo && A->ncrit == P->ncrit && A->nsurf == P->nsurf &&
        (A->precision == FMM_FP64) == (P->precision == FMM_FP64) && A->device == P->device && A->tree_mem &&
        A->tune.tile_split2 == P->tune.tile_split2 && A->tune.tile_split4 == P->tune.tile_split4 &&
        A->tune.work_cap_min == P->tune.work_cap_min && A->tune.work_cap_div == P->tune.work_cap_div &&
        A->tune.far_weight == P->tune.far_weight)
      return A;
  return nullptr;
}

// A live plan whose translation operators P can take: the same kernel,
// kappa, order and working type on a tree of the same points, root cube and
// ncrit (the operators depend on the level sizes and on the offsets the V
// lists use, not on the leaf items).
static fmm_plan *find_ops(const fmm_plan *P) {
  std::lock_guard<std::mutex> lock(g_tree_mu);
  for (fmm_plan *A : g_tree_plans)
    if (A->ops_mem && A->kernel == P->kernel && A->kappa == P->kappa && A->p == P->p &&
        A->tune.m2l_factored == P->tune.m2l_factored &&
        A->precision == P->precision && A->coord_hash == P->coord_hash && A->n == P->n &&
        A->mol_off == P->mol_off && A->W == P->W && A->mol_lo == P->mol_lo && A->ncrit == P->ncrit &&
        A->device == P->device && A->level_begin == P->level_begin && A->loff[1] == P->loff[1] &&
        A->lidx[1] == P->lidx[1])
      return A;
  return nullptr;
}

static void share_ops(fmm_plan *P, const fmm_plan *A) {
  P->ops_mem = A->ops_mem;
  P->pool1 = A->pool1; P->pool_bf = A->pool_bf;
  P->pool1_count = A->pool1_count; P->poolbf_count = A->poolbf_count;
  P->bf_kb = A->bf_kb;
  P->utu_id = A->utu_id; P->vsu_id = A->vsu_id; P->utd_id = A->utd_id; P->vsd_id = A->vsd_id;
  P->rank_u = A->rank_u; P->rank_d = A->rank_d;
  P->m2m_id = A->m2m_id; P->l2l_id = A->l2l_id; P->m2l_id = A->m2l_id;
  P->m2l_r_id = A->m2l_r_id; P->m2l_k = A->m2l_k; P->m2l_ldt = A->m2l_ldt;
  P->vs_alpha = A->vs_alpha; P->k_alpha = A->k_alpha;
  P->surf = A->surf;
  P->dt.box_geom = A->dt.box_geom;
  P->ops_shared = 1;
}

static void register_tree(fmm_plan *P) {
  if (!P->tree_mem) return;
  std::lock_guard<std::mutex> lock(g_tree_mu);
  g_tree_plans.push_back(P);
}

static void unregister_tree(fmm_plan *P) {
  std::lock_guard<std::mutex> lock(g_tree_mu);
  g_tree_plans.erase(std::remove(g_tree_plans.begin(), g_tree_plans.end(), P), g_tree_plans.end());
}

// P takes A's host tree and lists and A's read-only device buffers (sorted
// order, boxes, lists, leaf items, ranges); the sorted points (their fourth
// slot takes densities during an evaluation) and the split-tile partial
// sums are P's own.
static int share_tree(fmm_plan *P, const fmm_plan *A, hipStream_t s) {
  P->keys = A->keys; P->perm = A->perm;
  P->level = A->level; P->nchild = A->nchild; P->anchor = A->anchor; P->begin = A->begin; P->end = A->end;
  P->parent = A->parent; P->child_begin = A->child_begin; P->level_begin = A->level_begin; P->mol = A->mol;
  for (int k = 0; k < 4; ++k) { P->loff[k] = A->loff[k]; P->lidx[k] = A->lidx[k]; }
  P->leaf_ids = A->leaf_ids; P->vpair_src = A->vpair_src; P->vpair_tgt = A->vpair_tgt; P->p2l_boxes = A->p2l_boxes;
  P->p2p_inter = A->p2p_inter; P->far_inter = A->far_inter; P->item_pairs = A->item_pairs;
  P->tree_mem = A->tree_mem;
  P->dt = A->dt;
  P->dt.pts = nullptr;
  P->dt.parts = nullptr;
  P->dt.box_geom = nullptr;
  P->d_has_local = A->d_has_local; P->d_p2m_box = A->d_p2m_box; P->d_p2m_off = A->d_p2m_off;
  P->p2m_count = A->p2m_count;
  P->tree_on_device = A->tree_on_device;
  P->tree_shared = 1;
  const size_t es = P->precision == FMM_FP64 ? 8 : 4;
  int rc;
  if ((rc = dev_alloc(P, &P->dt.pts, (size_t)P->n * 4 * es))) return rc;
  FMM_HIP_TRY(hipMemcpyAsync(P->dt.pts, A->dt.pts, (size_t)P->n * 4 * es, hipMemcpyDeviceToDevice, s));
  if ((rc = dev_alloc(P, &P->dt.parts, std::max<size_t>(1, (size_t)P->dt.nparts) * MAX_NR * 4 * 64 * es))) return rc;
  return FMM_OK;
}

}  // namespace fmm

using namespace fmm;

extern "C" {

const char *fmm_last_error(void) { return g_err.c_str(); }

static int setup_common(const double *xyz_dev, const std::vector<int64_t> &off, int kernel, double kappa, int p,
                        int ncrit, int precision, fmm_stream_t stream, fmm_plan **out) {
  auto t0 = std::chrono::steady_clock::now();
  if (!out) { set_error("fmm_setup: out is NULL"); return FMM_EINVAL; }
  *out = nullptr;
  const int64_t n = off.back();
  if (n < 0 || n > 0x7fffffffll) { set_error("fmm_setup: n out of range"); return FMM_EINVAL; }
  if (n > 0 && !xyz_dev) { set_error("fmm_setup: xyz is NULL"); return FMM_EINVAL; }
  if (kernel != FMM_LAPLACE && kernel != FMM_YUKAWA) { set_error("fmm_setup: unknown kernel"); return FMM_EINVAL; }
  if (!(kappa >= 0.0) || !std::isfinite(kappa)) { set_error("fmm_setup: kappa must be finite and >= 0"); return FMM_EINVAL; }
  // p <= 10: the surface kernels hold one surface point per thread of a
  // workgroup of at most 512 (n_surf = 488 at p = 10)
  if (p < 2 || p > 10) { set_error("fmm_setup: p must be in [2, 10]"); return FMM_EINVAL; }
  if (ncrit < 1) { set_error("fmm_setup: ncrit must be >= 1"); return FMM_EINVAL; }
  if (precision != FMM_FP64 && precision != FMM_FP32 && precision != FMM_FP32_BF16X3) {
    set_error("fmm_setup: unknown precision");
    return FMM_EINVAL;
  }
  fmm_plan *P = new (std::nothrow) fmm_plan();
  if (!P) { set_error("fmm_setup: out of host memory"); return FMM_ENOMEM; }
  P->kernel = kernel; P->kappa = kernel == FMM_YUKAWA ? kappa : 0.0; P->p = p; P->ncrit = ncrit; P->precision = precision;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    P->tune = g_tune;
  }
  P->n = n;
  P->mol_off = off;
  P->nsurf = 6 * (p - 1) * (p - 1) + 2;
  P->ld = ((P->nsurf + 15) / 16) * 16;
  if (P->ld / 16 > 32) { delete P; set_error("fmm_setup: p too large for the GEMM kernel"); return FMM_EINVAL; }
  (void)hipGetDevice(&P->device);
  hipStream_t s = (hipStream_t)stream;
  const int nmol = (int)off.size() - 1;
  int rc = FMM_OK;
  auto tl = std::chrono::steady_clock::now();
  auto lap = [&](int stage) {  // time since the previous stage into setup_split[stage]
    const auto now = std::chrono::steady_clock::now();
    P->setup_split[stage] += std::chrono::duration<double, std::milli>(now - tl).count();
    tl = now;
  };
  do {
    if (n == 0) {
      P->level = {0}; P->nchild = {0}; P->anchor = {0, 0, 0}; P->begin = {0}; P->end = {0}; P->parent = {-1};
      P->child_begin = {-1}; P->level_begin = {0, 1}; P->mol = {0};
      for (int k = 0; k < 4; ++k) { P->loff[k] = {0, 0}; P->lidx[k].clear(); }
      P->dt.nbox = 1; P->dt.maxlevel = 0;
      break;
    }
    // per-molecule bounding boxes; one common root side W for the batch, so
    // that every molecule's tree has the same box sizes per level and the
    // translation operators are shared
    std::vector<double> cen(3 * nmol, 0.0);
    double ext = 0;
    for (int m = 0; m < nmol && !rc; ++m) {
      const int64_t nm = off[m + 1] - off[m];
      if (nm == 0) continue;
      double mn[3], mx[3];
      bool finite = true;
      uint64_t hm = 0;
      if ((rc = device_bbox(xyz_dev + 3 * off[m], nm, s, mn, mx, &finite, &hm))) break;
      // molecule m's coordinate checksum, tied to its index and size
      P->coord_hash = P->coord_hash * 0x100000001b3ull + (hm ^ ((uint64_t)m << 32) ^ (uint64_t)nm);
      if (!finite) { set_error("fmm_setup: non-finite coordinate"); rc = FMM_EINVAL; break; }
      for (int d = 0; d < 3; ++d) { cen[3 * m + d] = (mn[d] + mx[d]) * 0.5; ext = std::max(ext, mx[d] - mn[d]); }
    }
    if (rc) break;
    P->W = ext > 0 ? ext * (1.0 + std::ldexp(1.0, -20)) : 1.0;
    P->mol_lo.assign(3 * nmol, 0.0);
    for (int m = 0; m < nmol; ++m)
      for (int d = 0; d < 3; ++d) P->mol_lo[3 * m + d] = cen[3 * m + d] - 0.5 * P->W;
    for (int d = 0; d < 3; ++d) { P->lo[d] = P->mol_lo[d]; P->shift[d] = P->lo[d] + 0.5 * P->W; }
    if (fmm_plan *A = find_tree(P)) {
      // a live plan on the same points, ncrit, surface size and working
      // type: take its tree, lists and leaf items instead of building them
      if ((rc = share_tree(P, A, s))) break;
      lap(3);
    } else {
    P->tree_mem = std::make_shared<SharedAllocs>();
    uint64_t *d_keys = nullptr;
    if ((rc = device_morton_sort(xyz_dev, n, off, P->mol_lo, P->W, s, P->keys, P->perm, &d_keys))) break;
    lap(0);
    // octree levels and lists on the device; the host build remains for a
    // tree whose U/W traversal outgrows the device stack
    double ms_tree = 0, ms_lists = 0;
    const int trc = device_tree(P, d_keys, s, &ms_tree, &ms_lists);
    (void)hipFree(d_keys);
    if (trc < 0) { rc = trc; break; }
    lap(1);
    P->setup_split[1] -= ms_lists;
    P->setup_split[2] += ms_lists;
    P->tree_on_device = 1;
    if (trc == 1) {
      build_lists(P);
      P->tree_on_device = 0;
      lap(2);
    }
    // device tree (buffers shared with later plans on the same points)
    P->alloc_sink = &P->tree_mem->ptrs;
    std::vector<int32_t> perm32(n);
    for (int64_t i = 0; i < n; ++i) perm32[i] = (int32_t)P->perm[i];
    rc = upload(P, (void **)&P->dt.perm, perm32);
    P->alloc_sink = nullptr;
    if (rc) break;
    const size_t es = precision == FMM_FP64 ? 8 : 4;
    if ((rc = dev_alloc(P, &P->dt.pts, (size_t)n * 4 * es))) break;
    P->dt.n = n;
    {
      // points relative to their leaf's centre (the difference taken in FP64,
      // rounded once): single precision then resolves a pair's separation to
      // a fraction of a leaf width, wherever the molecule sits
      std::vector<int64_t> lb, le;
      std::vector<double> lsh;
      for (int64_t b = 0; b < (int64_t)P->level.size(); ++b) {
        if (P->nchild[b] || P->end[b] == P->begin[b]) continue;
        const int m = P->mol[b];
        const double sd = P->W / (double)(1ll << P->level[b]);
        lb.push_back(P->begin[b]);
        le.push_back(P->end[b]);
        for (int d = 0; d < 3; ++d)
          lsh.push_back(P->mol_lo[3 * m + d] + 0.5 * P->W + ((P->anchor[3 * b + d] + 0.5) * sd - 0.5 * P->W));
      }
      rc = device_gather_leaves(xyz_dev, P->dt.perm, lb, le, lsh, precision, P->dt.pts, s);
    }
    if (rc) break;
    P->alloc_sink = &P->tree_mem->ptrs;
    rc = upload_lists(P);
    P->alloc_sink = nullptr;
    if (rc) break;
    // per-plan scratch: partial sums of split leaf tiles
    if ((rc = dev_alloc(P, &P->dt.parts, std::max<size_t>(1, (size_t)P->dt.nparts) * MAX_NR * 4 * 64 * es))) break;
    lap(3);
    }
    P->tree_hash = tree_fingerprint(P);
    if (fmm_plan *A = find_ops(P)) {
      // a live plan of the same kernel, kappa, order and working type on the
      // same tree: its operators (they do not depend on the leaf items)
      share_ops(P, A);
    } else {
      P->ops_mem = std::make_shared<SharedAllocs>();
      P->alloc_sink = &P->ops_mem->ptrs;
      rc = precision == FMM_FP64 ? precompute_typed<double>(P) : precompute_typed<float>(P);
      P->alloc_sink = nullptr;
      if (rc) break;
    }
    hipError_t e = hipStreamSynchronize(s);
    lap(4);
    if (e != hipSuccess) { set_error(std::string("fmm_setup: ") + hipGetErrorString(e)); rc = FMM_EHIP; }
  } while (0);
  if (rc) { fmm_free(P); return rc; }
  P->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  register_tree(P);
  *out = P;
  return FMM_OK;
}

int fmm_setup(const double *xyz_dev, int64_t n, int kernel, double kappa, int p, int ncrit, int precision,
              fmm_stream_t stream, fmm_plan **out) {
  if (n < 0) { set_error("fmm_setup: n out of range"); if (out) *out = nullptr; return FMM_EINVAL; }
  return setup_common(xyz_dev, {0, n}, kernel, kappa, p, ncrit, precision, stream, out);
}

int fmm_setup_batch(const double *xyz_dev, const int64_t *offsets, int nmol, int kernel, double kappa, int p,
                    int ncrit, int precision, fmm_stream_t stream, fmm_plan **out) {
  if (out) *out = nullptr;
  if (nmol < 1 || !offsets) { set_error("fmm_setup_batch: need nmol >= 1 and offsets"); return FMM_EINVAL; }
  std::vector<int64_t> off(offsets, offsets + nmol + 1);
  if (off[0] != 0) { set_error("fmm_setup_batch: offsets[0] must be 0"); return FMM_EINVAL; }
  for (int m = 0; m < nmol; ++m)
    if (off[m + 1] < off[m]) { set_error("fmm_setup_batch: offsets must not decrease"); return FMM_EINVAL; }
  return setup_common(xyz_dev, off, kernel, kappa, p, ncrit, precision, stream, out);
}

int fmm_eval(fmm_plan *plan, const void *q_dev, int nrhs, void *pot_dev, void *grad_dev, fmm_stream_t stream) {
  if (!plan) { set_error("fmm_eval: plan is NULL"); return FMM_EINVAL; }
  if (nrhs < 1 || nrhs > 64) { set_error("fmm_eval: nrhs must be in [1, 64]"); return FMM_EINVAL; }
  if (plan->n == 0) return FMM_OK;
  if (!q_dev || !pot_dev) { set_error("fmm_eval: null buffer"); return FMM_EINVAL; }
  return eval_dispatch(plan, q_dev, nrhs, pot_dev, grad_dev, (hipStream_t)stream);
}

static bool shares_tree(const fmm_plan *A, const fmm_plan *B) {
  return A->kernel == FMM_LAPLACE && B->kernel == FMM_YUKAWA && A->tree_hash == B->tree_hash &&
         A->precision == B->precision && A->nsurf == B->nsurf && A->ncrit == B->ncrit && A->n == B->n &&
         A->dt.nitems == B->dt.nitems && A->dt.nparts == B->dt.nparts;
}

int fmm_eval_pair(fmm_plan *A, fmm_plan *B, const void *q_dev, int nrhs, void *pot_a, void *grad_a, void *pot_b,
                  void *grad_b, fmm_stream_t stream) {
  if (!A || !B) { set_error("fmm_eval_pair: plan is NULL"); return FMM_EINVAL; }
  if (A == B) { set_error("fmm_eval_pair: the two plans must differ"); return FMM_EINVAL; }
  if (A->n != B->n || (A->precision == FMM_FP64) != (B->precision == FMM_FP64)) {
    set_error("fmm_eval_pair: plans differ in point count or precision");
    return FMM_EINVAL;
  }
  if (nrhs < 1 || nrhs > 64) { set_error("fmm_eval_pair: nrhs must be in [1, 64]"); return FMM_EINVAL; }
  if (A->n == 0) return FMM_OK;
  if (!q_dev || !pot_a || !pot_b) { set_error("fmm_eval_pair: null buffer"); return FMM_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  const bool shared = shares_tree(A, B);
  if (!shared) {
    int rc;
    if ((rc = eval_dispatch(A, q_dev, nrhs, pot_a, grad_a, s))) return rc;
    return eval_dispatch(B, q_dev, nrhs, pot_b, grad_b, s);
  }
  return eval_pair_dispatch(A, B, q_dev, nrhs, pot_a, grad_a, pot_b, grad_b, s);
}

int fmm_eval_pair_md(fmm_plan *A, fmm_plan *B, const void *q_dev, const void *dip_dev, double qscale_a,
                     double qscale_b, void *pot_a, void *grad_a, void *pot_b, void *grad_b, fmm_stream_t stream) {
  if (!A || !B || A == B) { set_error("fmm_eval_pair_md: need two plans"); return FMM_EINVAL; }
  if (!shares_tree(A, B)) {
    set_error("fmm_eval_pair_md: plan_a must be a Laplace and plan_b a Yukawa plan on the same points, p, ncrit "
              "and precision");
    return FMM_EINVAL;
  }
  if (!std::isfinite(qscale_a) || !std::isfinite(qscale_b)) {
    set_error("fmm_eval_pair_md: non-finite charge scale");
    return FMM_EINVAL;
  }
  if (A->n == 0) return FMM_OK;
  if (!q_dev || !dip_dev || !pot_a || !pot_b) { set_error("fmm_eval_pair_md: null buffer"); return FMM_EINVAL; }
  return eval_pair_md_dispatch(A, B, q_dev, dip_dev, qscale_a, qscale_b, pot_a, grad_a, pot_b, grad_b,
                               (hipStream_t)stream);
}

int fmm_adjoint(fmm_plan *P, const void *q, const void *gbar, const void *gfwd, int nrhs, void *dq, void *dxyz,
                fmm_stream_t stream) {
  if (!P || !gbar || nrhs < 1 || nrhs > 64) { set_error("fmm_adjoint: bad argument"); return FMM_EINVAL; }
  if (dxyz && (!q || !gfwd)) { set_error("fmm_adjoint: position gradient needs q and the forward gradient"); return FMM_EINVAL; }
  if (P->n == 0) return FMM_OK;
  hipStream_t s = (hipStream_t)stream;
  const size_t es = P->precision == FMM_FP64 ? 8 : 4;
  const size_t need = (size_t)nrhs * P->n * 4 * es;  // psi + grad psi
  if (P->adj_bytes < need) {
    int rc;
    if ((rc = dev_alloc(P, &P->adj, need))) return rc;
    P->adj_bytes = need;
  }
  char *psi = (char *)P->adj;
  char *gpsi = psi + (size_t)nrhs * P->n * es;
  int rc;
  if ((rc = eval_dispatch(P, gbar, nrhs, psi, dxyz ? gpsi : nullptr, s))) return rc;
  if (dq) FMM_HIP_TRY(hipMemcpyAsync(dq, psi, (size_t)nrhs * P->n * es, hipMemcpyDeviceToDevice, s));
  if (dxyz) return adjoint_combine(P, nrhs, q, gbar, gfwd, gpsi, dxyz, s);
  return FMM_OK;
}

int fmm_info(const fmm_plan *P, fmm_info_t *o) {
  if (!P || !o) { set_error("fmm_info: null argument"); return FMM_EINVAL; }
  std::memset(o, 0, sizeof(*o));
  o->n_points = P->n;
  o->n_boxes = (int64_t)P->level.size();
  int64_t nl = 0;
  for (auto c : P->nchild) nl += c == 0;
  o->n_leaves = P->n ? nl : 0;
  o->max_level = (int32_t)P->level_begin.size() - 2;
  o->n_surf = P->nsurf;
  o->n_u_pairs = (int64_t)P->lidx[0].size();
  o->n_v_pairs = (int64_t)P->lidx[1].size();
  o->n_w_pairs = (int64_t)P->lidx[2].size();
  o->n_x_pairs = (int64_t)P->lidx[3].size();
  o->n_p2p_interactions = P->p2p_inter;
  o->device_bytes = P->device_bytes;
  o->setup_ms = P->setup_ms;
  o->n_far_interactions = P->far_inter;
  o->setup_sort_ms = P->setup_split[0];
  o->setup_tree_ms = P->setup_split[1];
  o->setup_lists_ms = P->setup_split[2];
  o->setup_items_ms = P->setup_split[3];
  o->setup_ops_ms = P->setup_split[4];
  o->tree_on_device = P->tree_on_device;
  o->tree_shared = P->tree_shared;
  const int nit = (int)P->item_pairs.size();
  o->n_items = nit;
  o->n_items_early = near_early_items(P->tune, nit, P->dt.maxlevel >= 2);
  for (int i = nit - o->n_items_early; i < nit; ++i) o->n_p2p_early += P->item_pairs[i];
  if (P->chain_ctr && P->chain_ctr_n > 0) {
    int32_t e = 0;
    FMM_HIP_TRY(hipDeviceSynchronize());
    FMM_HIP_TRY(hipMemcpy(&e, P->chain_ctr + P->chain_ctr_n - 1, sizeof(e), hipMemcpyDeviceToHost));
    o->chain_timeouts = e;
  }
  for (size_t l = 0; l < P->rank_u.size(); ++l) o->rank_up = std::max(o->rank_up, (int32_t)P->rank_u[l]);
  for (size_t l = 0; l < P->rank_d.size(); ++l) o->rank_down = std::max(o->rank_down, (int32_t)P->rank_d[l]);
  return FMM_OK;
}

int fmm_get_tree(const fmm_plan *P, int64_t *perm, int64_t *keys, int32_t *level, int64_t *anchor_xyz,
                 int64_t *begin, int64_t *end, int64_t *parent, int64_t *child_begin, int32_t *nchild,
                 int64_t *list_off, int64_t *list_idx) {
  if (!P) { set_error("fmm_get_tree: plan is NULL"); return FMM_EINVAL; }
  const size_t nb = P->level.size();
  if (perm) std::copy(P->perm.begin(), P->perm.end(), perm);
  if (keys) std::copy(P->keys.begin(), P->keys.end(), keys);
  if (level) std::copy(P->level.begin(), P->level.end(), level);
  if (anchor_xyz) std::copy(P->anchor.begin(), P->anchor.end(), anchor_xyz);
  if (begin) std::copy(P->begin.begin(), P->begin.end(), begin);
  if (end) std::copy(P->end.begin(), P->end.end(), end);
  if (parent) std::copy(P->parent.begin(), P->parent.end(), parent);
  if (child_begin) std::copy(P->child_begin.begin(), P->child_begin.end(), child_begin);
  if (nchild) std::copy(P->nchild.begin(), P->nchild.end(), nchild);
  int64_t base = 0;
  for (int k = 0; k < 4; ++k) {
    if (list_off)
      for (size_t b = 0; b <= nb; ++b) list_off[k * (nb + 1) + b] = base + P->loff[k][b];
    if (list_idx) std::copy(P->lidx[k].begin(), P->lidx[k].end(), list_idx + base);
    base += (int64_t)P->lidx[k].size();
  }
  return FMM_OK;
}

int fmm_get_root(const fmm_plan *P, double *lo3, double *width) {
  if (!P) { set_error("fmm_get_root: plan is NULL"); return FMM_EINVAL; }
  if (lo3) for (int d = 0; d < 3; ++d) lo3[d] = P->lo[d];
  if (width) *width = P->W;
  return FMM_OK;
}

int fmm_set_tuning(const fmm_tuning_t *t) {
  if (!t) { set_error("fmm_set_tuning: null argument"); return FMM_EINVAL; }
  if (t->tile_split2 < 0 || t->tile_split2 > 32 || t->tile_split4 < 0 || t->tile_split4 > 16 ||
      t->work_cap_min < 1 || t->work_cap_div < 1 || !(t->far_weight > 0.0) || !std::isfinite(t->far_weight) ||
      t->gemm_rbw < 0 || t->gemm_rbw > 8 || t->m2l_factored < 0 || t->m2l_factored > 1 || t->pair_order < 0 ||
      t->pair_order > 4 || t->near_lds < 0 || t->near_lds > 65536 ||
      t->gemm_lat < 0 || t->gemm_lat > (1 << 20) || t->gemm_chain < 0 || t->gemm_chain > 1 ||
      (t->m2l_cols != 64 && t->m2l_cols != 128) || t->gemm_narrow < 0 || t->gemm_narrow > 1 ||
      t->near_early < 0 || t->near_early > 900 || t->near_early_grid < 64 || t->near_early_grid > 65536 ||
      t->m2l_early < 0 || t->m2l_early > 1 || t->near_early_start < 0 || t->near_early_start > 1) {
    set_error("fmm_set_tuning: value out of range");
    return FMM_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune = *t;
  return FMM_OK;
}

int fmm_get_tuning(fmm_tuning_t *t) {
  if (!t) { set_error("fmm_get_tuning: null argument"); return FMM_EINVAL; }
  std::lock_guard<std::mutex> lock(g_tune_mu);
  *t = g_tune;
  return FMM_OK;
}

int fmm_set_profiling(fmm_plan *P, int enable) {
  if (!P) { set_error("fmm_set_profiling: plan is NULL"); return FMM_EINVAL; }
  P->profiling = enable & (((1 << FMM_PHASE_COUNT) - 1) | FMM_PROFILE_SERIAL);
  return FMM_OK;
}

int fmm_get_phase_times(fmm_plan *P, double *ms, int64_t *launches, int nphase) {
  if (!P || nphase < 0 || nphase > FMM_PHASE_COUNT) { set_error("fmm_get_phase_times: bad argument"); return FMM_EINVAL; }
  std::vector<double> acc(FMM_PHASE_COUNT, 0.0);
  std::vector<int64_t> cnt(FMM_PHASE_COUNT, 0);
  for (auto &pe : P->prof_events) {
    FMM_HIP_TRY(hipEventSynchronize(pe.second.second));
    float t = 0;
    FMM_HIP_TRY(hipEventElapsedTime(&t, pe.second.first, pe.second.second));
    acc[pe.first] += t;
    cnt[pe.first] += 1;
    P->event_pool.push_back(pe.second.first);
    P->event_pool.push_back(pe.second.second);
  }
  P->prof_events.clear();
  for (int i = 0; i < nphase; ++i) {
    if (ms) ms[i] = acc[i];
    if (launches) launches[i] = cnt[i];
  }
  return FMM_OK;
}

void fmm_free(fmm_plan *P) {
  if (!P) return;
  unregister_tree(P);
  for (auto &pe : P->prof_events) { (void)hipEventDestroy(pe.second.first); (void)hipEventDestroy(pe.second.second); }
  for (hipEvent_t e : P->event_pool) (void)hipEventDestroy(e);
  for (hipStream_t st : {P->aux, P->aux2, P->aux3})  // the device's shared side streams: wait, keep
    if (st) (void)hipStreamSynchronize(st);
  for (hipEvent_t e : {P->ev_fork, P->ev_join, P->ev_up, P->ev_m2l, P->ev_near, P->ev_m2m, P->ev_m2lf})
    if (e) (void)hipEventDestroy(e);
  for (void *p : P->allocs) (void)hipFree(p);
  delete P;
}

}  // extern "C"

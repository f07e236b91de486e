// HIP kernels of the kernel-independent FMM for gfx950 (MI355X) and the
// evaluation driver behind fmm_eval.
//
// Pass order (Methods, Fast multipole method): P2M at the leaves, M2M
// bottom-up, M2L (plus P2L for X-list boxes), L2L top-down, then at every
// leaf L2P, M2P (W list) and P2P (U list).  All dense translations
// (UC2E after P2M, M2M, M2L, L2L, DC2E) run through one gather-GEMM kernel on
// MFMA; the point-kernel stages (P2P/L2P/M2P and P2M/P2L) run on the VALU
// with sources staged through LDS.
//
// Kernel arithmetic: every kernel evaluation omits the 1/(4 pi) of the
// Green's functions (the matching equations are invariant to it); the final
// write multiplies by 1/(4 pi).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include "fmm_internal.h"

namespace fmm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = floatx4; };
template <> struct Vec4<double> { using type = doublex4; };

__device__ inline floatx4 mfma_16x16x4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline doublex4 mfma_16x16x4(double a, double b, doublex4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline float dev_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
// FP64 reciprocal square root: the hardware estimate refined by two
// Newton-Raphson steps for 1/sqrt(x), y <- y (3/2 - (x/2) y^2), each of which
// doubles the number of correct bits (the estimate's ~2^-22 relative error
// becomes a few ulp); x = 0 gives inf like 1/sqrt(0).
__device__ inline double dev_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  if (!(x > 0.0) || !(y < 1.0e300)) return y;
  const double h = 0.5 * x;
  y = y * fma(-h, y * y, 1.5);
  y = y * fma(-h, y * y, 1.5);
  return y;
}
__device__ inline float dev_exp(float x) { return __expf(x); }
__device__ inline double dev_exp(double x) { return exp(x); }
__device__ inline float dev_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ inline double dev_exp2(double x) { return exp2(x); }

// ---------------------------------------------------------------------------
// Setup helpers: bounding box, Morton keys, point gather.
// ---------------------------------------------------------------------------
// splitmix64 finaliser (a bijective 64-bit mix)
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Per block: the coordinate minima and maxima (NaN minimum when a coordinate
// is not finite) and a checksum of the coordinates' bit patterns at their
// positions (wrapping sum over points of a mix of index and bits; integer
// addition, so the total does not depend on the order of the sum).  part
// holds 7 doubles per block: 3 minima, 3 maxima, the checksum's bits.
__global__ void k_bbox_partial(const double *__restrict__ xyz, int64_t n, double *__restrict__ part) {
  __shared__ double smin[3][256], smax[3][256];
  __shared__ unsigned long long shash[256];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  int bad = 0;
  uint64_t hsum = 0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    uint64_t h = mix64((uint64_t)i + 0x9e3779b97f4a7c15ull);
    for (int d = 0; d < 3; ++d) {
      double v = xyz[i * 3 + d];
      if (!isfinite(v)) bad = 1;
      mn[d] = fmin(mn[d], v);
      mx[d] = fmax(mx[d], v);
      h = mix64(h ^ (uint64_t)__double_as_longlong(v));
    }
    hsum += h;
  }
  shash[threadIdx.x] = hsum;
  if (bad) { mn[0] = NAN; }
  for (int d = 0; d < 3; ++d) { smin[d][threadIdx.x] = mn[d]; smax[d][threadIdx.x] = mx[d]; }
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      for (int d = 0; d < 3; ++d) {
        double a = smin[d][threadIdx.x], b = smin[d][threadIdx.x + s];
        smin[d][threadIdx.x] = (isnan(a) || isnan(b)) ? NAN : fmin(a, b);
        smax[d][threadIdx.x] = fmax(smax[d][threadIdx.x], smax[d][threadIdx.x + s]);
      }
      shash[threadIdx.x] += shash[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int d = 0; d < 3; ++d) { part[blockIdx.x * 7 + d] = smin[d][0]; part[blockIdx.x * 7 + 3 + d] = smax[d][0]; }
    part[blockIdx.x * 7 + 6] = __longlong_as_double((long long)shash[0]);
  }
}

__device__ inline uint64_t spread3(uint64_t v) {
  v &= 0x1fffff;
  v = (v | v << 32) & 0x1f00000000ffffull;
  v = (v | v << 16) & 0x1f0000ff0000ffull;
  v = (v | v << 8) & 0x100f00f00f00f00full;
  v = (v | v << 4) & 0x10c30c30c30c30c3ull;
  v = (v | v << 2) & 0x1249249249249249ull;
  return v;
}

__global__ void k_morton(const double *__restrict__ xyz, int64_t n, double lox, double loy, double loz,
                         double W, uint64_t *__restrict__ keys, int32_t *__restrict__ idx, int64_t base) {
  int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= n) return;
  const double lo[3] = {lox, loy, loz};
  uint64_t c[3];
  for (int d = 0; d < 3; ++d) {
    double t = (xyz[i * 3 + d] - lo[d]) / W;
    double f = floor(t * 2097152.0);
    f = f < 0.0 ? 0.0 : (f > 2097151.0 ? 2097151.0 : f);
    c[d] = (uint64_t)f;
  }
  keys[i] = (spread3(c[0]) << 2) | (spread3(c[1]) << 1) | spread3(c[2]);
  idx[i] = (int32_t)(base + i);
}

// One workgroup per leaf: its sorted points minus the leaf's absolute centre
// (lsh), in FP64, rounded once to T.
template <typename T>
__global__ void k_gather_leaves(const double *__restrict__ xyz, const int32_t *__restrict__ perm,
                                const int64_t *__restrict__ lb, const int64_t *__restrict__ le,
                                const double *__restrict__ lsh, T *__restrict__ pts) {
  const int leaf = blockIdx.x;
  const double sx = lsh[3 * leaf], sy = lsh[3 * leaf + 1], sz = lsh[3 * leaf + 2];
  for (int64_t i = lb[leaf] + threadIdx.x; i < le[leaf]; i += blockDim.x) {
    const int64_t j = perm[i];
    pts[i * 4 + 0] = (T)(xyz[j * 3 + 0] - sx);
    pts[i * 4 + 1] = (T)(xyz[j * 3 + 1] - sy);
    pts[i * 4 + 2] = (T)(xyz[j * 3 + 2] - sz);
    pts[i * 4 + 3] = (T)0;
  }
}

int device_bbox(const double *xyz, int64_t n, hipStream_t s, double mn[3], double mx[3], bool *finite,
                uint64_t *hash) {
  int nb = (int)std::min<int64_t>(1024, (n + 255) / 256);
  double *part = nullptr;
  FMM_HIP_TRY(hipMalloc(&part, sizeof(double) * 7 * nb));
  hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(256), 0, s, xyz, n, part);
  std::vector<double> h(7 * nb);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), part, sizeof(double) * 7 * nb, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(part);
  if (e != hipSuccess) { set_error(std::string("bbox: ") + hipGetErrorString(e)); return FMM_EHIP; }
  *finite = true;
  for (int d = 0; d < 3; ++d) { mn[d] = INFINITY; mx[d] = -INFINITY; }
  uint64_t hs = 0;
  for (int b = 0; b < nb; ++b) {
    for (int d = 0; d < 3; ++d) {
      double a = h[b * 7 + d], c = h[b * 7 + 3 + d];
      if (std::isnan(a) || std::isinf(a) || std::isinf(c)) *finite = false;
      mn[d] = std::min(mn[d], a);
      mx[d] = std::max(mx[d], c);
    }
    uint64_t hb;
    std::memcpy(&hb, &h[b * 7 + 6], 8);
    hs += hb;
  }
  if (hash) *hash = hs;
  return FMM_OK;
}

// Morton keys (each molecule in its own root cube of side W, lower corner
// lo[3m..3m+2]) and a stable radix sort within each molecule's range; the
// sorted keys and the permutation (global indices) come back to the host,
// and with keys_dev the device copy of the sorted keys is kept (the caller
// frees it).
int device_morton_sort(const double *xyz, int64_t n, const std::vector<int64_t> &off, const std::vector<double> &lo,
                       double W, hipStream_t s, std::vector<int64_t> &keys_out, std::vector<int64_t> &perm_out,
                       uint64_t **keys_dev) {
  const int nmol = (int)off.size() - 1;
  uint64_t *k0 = nullptr, *k1 = nullptr;
  int32_t *v0 = nullptr, *v1 = nullptr;
  int64_t *d_off = nullptr;
  void *tmp = nullptr;
  size_t tmp_bytes = 0;
  int rc = FMM_OK;
  auto fail = [&](const char *what, hipError_t e) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    rc = FMM_EHIP;
  };
  hipError_t e;
  if ((e = hipMalloc(&k0, n * 8)) != hipSuccess || (e = hipMalloc(&k1, n * 8)) != hipSuccess ||
      (e = hipMalloc(&v0, n * 4)) != hipSuccess || (e = hipMalloc(&v1, n * 4)) != hipSuccess ||
      (e = hipMalloc(&d_off, (nmol + 1) * 8)) != hipSuccess) {
    fail("morton alloc", e);
  } else {
    for (int m = 0; m < nmol; ++m) {
      const int64_t nm = off[m + 1] - off[m];
      if (nm == 0) continue;
      hipLaunchKernelGGL(k_morton, dim3((unsigned)((nm + 255) / 256)), dim3(256), 0, s, xyz + 3 * off[m], nm,
                         lo[3 * m], lo[3 * m + 1], lo[3 * m + 2], W, k0 + off[m], v0 + off[m], off[m]);
    }
    e = hipMemcpyAsync(d_off, off.data(), (nmol + 1) * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      if (nmol == 1) {
        e = rocprim::radix_sort_pairs(nullptr, tmp_bytes, k0, k1, v0, v1, (size_t)n, 0, 63, s);
        if (e == hipSuccess) e = hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 16));
        if (e == hipSuccess) e = rocprim::radix_sort_pairs(tmp, tmp_bytes, k0, k1, v0, v1, (size_t)n, 0, 63, s);
      } else {
        e = rocprim::segmented_radix_sort_pairs(nullptr, tmp_bytes, k0, k1, v0, v1, (unsigned)n, (unsigned)nmol, d_off,
                                                d_off + 1, 0, 63, s);
        if (e == hipSuccess) e = hipMalloc(&tmp, std::max<size_t>(tmp_bytes, 16));
        if (e == hipSuccess)
          e = rocprim::segmented_radix_sort_pairs(tmp, tmp_bytes, k0, k1, v0, v1, (unsigned)n, (unsigned)nmol, d_off,
                                                  d_off + 1, 0, 63, s);
      }
    }
    std::vector<uint64_t> hk(n);
    std::vector<int32_t> hv(n);
    if (e == hipSuccess) e = hipMemcpyAsync(hk.data(), k1, n * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hv.data(), v1, n * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) fail("morton sort", e);
    else {
      keys_out.resize(n);
      perm_out.resize(n);
      for (int64_t i = 0; i < n; ++i) { keys_out[i] = (int64_t)hk[i]; perm_out[i] = hv[i]; }
    }
  }
  // the sorted keys stay on the device for the tree build when asked for
  if (keys_dev && rc == FMM_OK) {
    *keys_dev = k1;
    k1 = nullptr;
  }
  (void)hipFree(k0); (void)hipFree(k1); (void)hipFree(v0); (void)hipFree(v1); (void)hipFree(tmp); (void)hipFree(d_off);
  return rc;
}

int device_gather_leaves(const double *xyz, const int32_t *perm, const std::vector<int64_t> &lb,
                         const std::vector<int64_t> &le, const std::vector<double> &lsh, int prec, void *pts,
                         hipStream_t s) {
  const size_t nl = lb.size();
  if (nl == 0) return FMM_OK;
  int64_t *d_lb = nullptr, *d_le = nullptr;
  double *d_sh = nullptr;
  hipError_t e = hipMalloc(&d_lb, nl * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(&d_le, nl * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(&d_sh, nl * 3 * sizeof(double));
  if (e == hipSuccess) e = hipMemcpyAsync(d_lb, lb.data(), nl * sizeof(int64_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_le, le.data(), nl * sizeof(int64_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_sh, lsh.data(), nl * 3 * sizeof(double), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    if (prec == FMM_FP64)
      hipLaunchKernelGGL(k_gather_leaves<double>, dim3((unsigned)nl), dim3(128), 0, s, xyz, perm, d_lb, d_le, d_sh,
                         (double *)pts);
    else
      hipLaunchKernelGGL(k_gather_leaves<float>, dim3((unsigned)nl), dim3(128), 0, s, xyz, perm, d_lb, d_le, d_sh,
                         (float *)pts);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d_lb);
  (void)hipFree(d_le);
  (void)hipFree(d_sh);
  if (e != hipSuccess) {
    set_error(std::string("gather: ") + hipGetErrorString(e));
    return FMM_EHIP;
  }
  return FMM_OK;
}

// ---------------------------------------------------------------------------
// Gather-GEMM on MFMA:  Y[dst[c]] (op)= alpha * A * concat_s X[src[c*S+s]]
// One workgroup (4 waves) computes all ld rows of a 64-column tile.  A is
// pre-swizzled so that each lane loads the A operands of four consecutive
// 16x16x4 MFMA k-steps with one 4-element vector load; B (the gathered
// columns) is staged through LDS 64 k-values at a time.
// Each wave owns RBW consecutive 16-row blocks and all four 16-column blocks.
// ---------------------------------------------------------------------------
// Workgroups are dealt to the eight XCDs round robin (workgroup b runs on XCD
// b % 8), each with its own L2.  Task lists keep the columns that share a
// matrix in consecutive tasks; mapping workgroup b to task
// (b % 8) * per + b / 8 gives every XCD one contiguous run of tasks, so a
// matrix is fetched into one L2 rather than into all eight.  The grid is
// 8 * per workgroups; those past the last task return at once.
__device__ inline int xcd_task() {
  const int per = (int)(gridDim.x >> 3);
  return (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
}

// Workgroup -> (batch, task): the first 8 * ceil(ntask0 / 8) workgroups
// serve batch 0, the rest batch 1, each with the XCD-contiguous mapping.
__device__ inline bool gemm_pick(const GemmArgs &g0, const GemmArgs &g1, GemmArgs &g, int &task) {
  const int per0 = (g0.ntask + 7) >> 3;
  int b = (int)blockIdx.x;
  const bool second = b >= 8 * per0;
  g = second ? g1 : g0;
  if (second) b -= 8 * per0;
  const int per = (g.ntask + 7) >> 3;
  task = (b & 7) * per + (b >> 3);
  return task < g.ntask;
}

template <typename T, int RBW>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g0, GemmArgs g1) {
  // Raised wave priority for instruction issue: in a pair evaluation the
  // GEMM passes share each SIMD with near-field waves that could issue VALU
  // work every cycle, and the passes are on the evaluation's critical path
  // (+1.3% per pair step, measured A/B on one device).  The same in
  // k_gemm_bf3 and k_pair_reduce.
  __builtin_amdgcn_s_setprio(3);
  // g.S segments of g.seg k-values per column (segment s of column c is row
  // src[c*S+s] of X, row length g.ldx); g.KQ: 16-wide k groups per stored
  // row block of A; g.klen: k-values read; g.nrb: 16-row blocks computed
  // (a task's nrb and klen, when set, are smaller: the M2L ranks of its
  // level);
  // output rows have length g.ldy.
  using V4 = typename Vec4<T>::type;
  GemmArgs g;
  int task;
  if (!gemm_pick(g0, g1, g, task)) return;
  const GemmTask tk = g.tasks[task];
  const int S = g.S, seg = g.seg, KQ = g.KQ, ld = g.ldx, ldy = g.ldy, mode = g.mode;
  const int nrb = tk.nrb > 0 ? min(tk.nrb, g.nrb) : g.nrb;
  const int K = tk.klen > 0 ? min(tk.klen, g.klen) : g.klen;
  const int32_t *__restrict__ src = g.src;
  const int32_t *__restrict__ dst = g.dst;
  const T *__restrict__ X = (const T *)g.X;
  T *__restrict__ Y = (T *)g.Y;
  const int KQK = K >> 4;         // k-groups actually read
  const T *__restrict__ A = (const T *)g.pool + (int64_t)tk.mat * g.mstride;
  __shared__ T Bs[64][GEMM_NT + 1];
  __shared__ int32_t s_src[GEMM_NT * 8];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = (int)blockIdx.y * 4 + (tid >> 6);  // row-block group of this wave
  for (int i = tid; i < GEMM_NT * S; i += 256) {
    int c = i / S;
    s_src[i] = (c < tk.ncol) ? src[(int64_t)(tk.col0 + c) * S + (i - c * S)] : -1;
  }
  V4 acc[RBW][4];
#pragma unroll
  for (int r = 0; r < RBW; ++r)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[r][cb] = V4{0, 0, 0, 0};
  __syncthreads();
  const int scol = tid >> 2, spart = (tid & 3) * 16;
  for (int kc = 0; kc < K; kc += 64) {
    {
      T vals[16];
      const int k0 = kc + spart;
      int row = -1, kk = 0;
      if (k0 < K) {
        int sg = k0 / seg;
        kk = k0 - sg * seg;
        row = s_src[scol * S + sg];
      }
      if (row >= 0) {
        const V4 *p = reinterpret_cast<const V4 *>(X + (int64_t)row * ld + kk);
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          V4 v = p[q4];
          vals[q4 * 4 + 0] = v[0]; vals[q4 * 4 + 1] = v[1]; vals[q4 * 4 + 2] = v[2]; vals[q4 * 4 + 3] = v[3];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) vals[e] = (T)0;
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) Bs[spart + e][scol] = vals[e];
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < 4; ++kq) {
      const int gkq = (kc >> 4) + kq;
      if (gkq < KQK) {
        V4 a[RBW];
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
          const int rb = wave * RBW + r;
          if (rb < nrb) a[r] = *reinterpret_cast<const V4 *>(A + ((int64_t)(rb * KQ + gkq) * 64 + lane) * 4);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int kl = (kq * 4 + t) * 4 + (lane >> 4);
          T b[4];
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) b[cb] = Bs[kl][cb * 16 + (lane & 15)];
#pragma unroll
          for (int r = 0; r < RBW; ++r) {
            if (wave * RBW + r < nrb) {
#pragma unroll
              for (int cb = 0; cb < 4; ++cb) acc[r][cb] = mfma_16x16x4(a[r][t], b[cb], acc[r][cb]);
            }
          }
        }
      }
    }
    __syncthreads();
  }
  const T alpha = (T)tk.alpha;
#pragma unroll
  for (int r = 0; r < RBW; ++r) {
    const int rb = wave * RBW + r;
    if (rb >= nrb) continue;
    const int i0 = rb * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int c = cb * 16 + (lane & 15);
      if (c >= tk.ncol) continue;
      const int64_t row = dst[tk.col0 + c];
      T *y = Y + row * ldy + i0;
      V4 v = acc[r][cb] * alpha;
      if (mode == GEMM_STORE) {
        *reinterpret_cast<V4 *>(y) = v;
      } else {
        V4 o = *reinterpret_cast<V4 *>(y);
        *reinterpret_cast<V4 *>(y) = o + v;
      }
    }
  }
}

// One wave per (64-column task, 16-row block), for the passes that run beside
// the near field: a 64-thread workgroup with few registers fits beside the
// near field's waves as they retire, where a 256-thread one waits for a whole
// compute unit's worth of them.  Each wave stages its own 64 columns (lane c
// loads column c) to LDS; the MFMAs run in k_gemm's k order, so the results
// are the same bit for bit.
template <typename T>
__global__ __launch_bounds__(64) void k_gemm_narrow(GemmArgs g0, GemmArgs g1) {
  __builtin_amdgcn_s_setprio(3);
  using V4 = typename Vec4<T>::type;
  GemmArgs g;
  int task;
  if (!gemm_pick(g0, g1, g, task)) return;
  const GemmTask tk = g.tasks[task];
  const int nrb = tk.nrb > 0 ? min(tk.nrb, g.nrb) : g.nrb;
  const int rb = (int)blockIdx.y;
  if (rb >= nrb) return;
  const int S = g.S, seg = g.seg, KQ = g.KQ, ld = g.ldx, ldy = g.ldy, mode = g.mode;
  const int K = tk.klen > 0 ? min(tk.klen, g.klen) : g.klen;
  const int KQK = K >> 4;
  const int32_t *__restrict__ src = g.src;
  const T *__restrict__ X = (const T *)g.X;
  T *__restrict__ Y = (T *)g.Y;
  const int lane = threadIdx.x;
  const T *__restrict__ A = (const T *)g.pool + (int64_t)tk.mat * g.mstride + ((int64_t)rb * KQ * 64 + lane) * 4;
  __shared__ T Bs[64][GEMM_NT + 1];
  V4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = V4{0, 0, 0, 0};
  for (int kc = 0; kc < K; kc += 64) {
#pragma unroll 4
    for (int q = 0; q < 16; ++q) {
      const int k0 = kc + q * 4;
      V4 v = V4{0, 0, 0, 0};
      if (lane < tk.ncol && k0 < K) {
        const int sg = k0 / seg, kk = k0 - sg * seg;
        const int row = src[(int64_t)(tk.col0 + lane) * S + sg];
        if (row >= 0) v = *reinterpret_cast<const V4 *>(X + (int64_t)row * ld + kk);
      }
      Bs[q * 4 + 0][lane] = v[0];
      Bs[q * 4 + 1][lane] = v[1];
      Bs[q * 4 + 2][lane] = v[2];
      Bs[q * 4 + 3][lane] = v[3];
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < 4; ++kq) {
      const int gkq = (kc >> 4) + kq;
      if (gkq < KQK) {
        const V4 a = *reinterpret_cast<const V4 *>(A + (int64_t)gkq * 256);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int kl = (kq * 4 + t) * 4 + (lane >> 4);
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) acc[cb] = mfma_16x16x4(a[t], Bs[kl][cb * 16 + (lane & 15)], acc[cb]);
        }
      }
    }
    __syncthreads();
  }
  const T alpha = (T)tk.alpha;
  const int i0 = rb * 16 + 4 * (lane >> 4);
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int c = cb * 16 + (lane & 15);
    if (c >= tk.ncol) continue;
    T *y = Y + (int64_t)g.dst[tk.col0 + c] * ldy + i0;
    const V4 r = acc[cb] * alpha;
    if (mode == GEMM_STORE) {
      *reinterpret_cast<V4 *>(y) = r;
    } else {
      V4 o = *reinterpret_cast<V4 *>(y);
      *reinterpret_cast<V4 *>(y) = o + r;
    }
  }
}

// Latency-bound launches (fewer workgroups than the device has compute
// units: the M2M and L2L levels, the surface projections): the same
// gather-GEMM with one 16-row block per wave, every A fragment of the wave
// loaded before the first MFMA and the whole K extent (KCH 64-wide chunks)
// of the 64 gathered columns staged to LDS at once, so that a workgroup
// waits for memory once instead of once per chunk.  The MFMAs run in the
// same k order as k_gemm, so the results are the same bit for bit.
template <typename T, int KCH>
__device__ __forceinline__ void gemm_lat_tile(const GemmArgs &g, int task, int yg) {
  using V4 = typename Vec4<T>::type;
  const GemmTask tk = g.tasks[task];
  const int S = g.S, seg = g.seg, KQ = g.KQ, ld = g.ldx, ldy = g.ldy, mode = g.mode;
  const int nrb = tk.nrb > 0 ? min(tk.nrb, g.nrb) : g.nrb;
  const int K = tk.klen > 0 ? min(tk.klen, g.klen) : g.klen;  // <= 64 KCH (checked by the launcher)
  const int KQK = K >> 4;
  const int32_t *__restrict__ src = g.src;
  const int32_t *__restrict__ dst = g.dst;
  const T *__restrict__ X = (const T *)g.X;
  T *__restrict__ Y = (T *)g.Y;
  __shared__ T Bs[64 * KCH][GEMM_NT + 1];
  __shared__ int32_t s_src[GEMM_NT * 8];
  const int tid = threadIdx.x, lane = tid & 63;
  const int rb = yg * 4 + (tid >> 6);  // this wave's row block
  const bool live = rb < nrb;
  const T *__restrict__ A = (const T *)g.pool + (int64_t)tk.mat * g.mstride + ((int64_t)rb * KQ * 64 + lane) * 4;
  V4 a[4 * KCH];
#pragma unroll
  for (int q = 0; q < 4 * KCH; ++q) a[q] = (live && q < KQK) ? *reinterpret_cast<const V4 *>(A + (int64_t)q * 256) : V4{0, 0, 0, 0};
  for (int i = tid; i < GEMM_NT * S; i += 256) {
    int c = i / S;
    s_src[i] = (c < tk.ncol) ? src[(int64_t)(tk.col0 + c) * S + (i - c * S)] : -1;
  }
  __syncthreads();
  const int scol = tid >> 2, spart = (tid & 3) * 16;
  V4 v[KCH][4];
#pragma unroll
  for (int ch = 0; ch < KCH; ++ch) {
    const int k0 = ch * 64 + spart;
    int row = -1, kk = 0;
    if (k0 < K) {
      const int sg = k0 / seg;
      kk = k0 - sg * seg;
      row = s_src[scol * S + sg];
    }
    const V4 *p = reinterpret_cast<const V4 *>(X + (int64_t)(row >= 0 ? row : 0) * ld + kk);
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) v[ch][q4] = row >= 0 ? p[q4] : V4{0, 0, 0, 0};
  }
#pragma unroll
  for (int ch = 0; ch < KCH; ++ch)
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
      for (int e = 0; e < 4; ++e) Bs[ch * 64 + spart + q4 * 4 + e][scol] = v[ch][q4][e];
  __syncthreads();
  if (!live) return;
  V4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = V4{0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 4 * KCH; ++q) {
    if (q < KQK) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int kl = (q * 4 + t) * 4 + (lane >> 4);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = mfma_16x16x4(a[q][t], Bs[kl][cb * 16 + (lane & 15)], acc[cb]);
      }
    }
  }
  const T alpha = (T)tk.alpha;
  const int i0 = rb * 16 + 4 * (lane >> 4);
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int c = cb * 16 + (lane & 15);
    if (c >= tk.ncol) continue;
    const int64_t row = dst[tk.col0 + c];
    T *y = Y + row * ldy + i0;
    V4 r = acc[cb] * alpha;
    if (mode == GEMM_STORE) {
      *reinterpret_cast<V4 *>(y) = r;
    } else {
      V4 o = *reinterpret_cast<V4 *>(y);
      *reinterpret_cast<V4 *>(y) = o + r;
    }
  }
}

template <typename T, int KCH>
__global__ __launch_bounds__(256) void k_gemm_lat(GemmArgs g0, GemmArgs g1) {
  __builtin_amdgcn_s_setprio(3);
  GemmArgs g;
  int task;
  if (!gemm_pick(g0, g1, g, task)) return;
  gemm_lat_tile<T, KCH>(g, task, (int)blockIdx.y);
}

// ---------------------------------------------------------------------------
// The same gather-GEMM with each FP32 operand split into bf16 high and low
// parts (x = hi + lo, hi = bf16(x), lo = bf16(x - hi)) and three
// 16x16x32 bf16 MFMAs per 32-wide k step (hi*hi + hi*lo + lo*hi), FP32
// accumulation.  A is pre-split and swizzled (per 16-row block and 32-wide k
// block, 64 lanes x 8 bf16 for hi, then for lo); B is split while it is
// staged to LDS, stored column-major so that each lane reads its 8
// consecutive k values with one 16-byte LDS load.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ inline unsigned short f2bf_rne(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

template <int RBW, int NT = GEMM_NT>
__global__ __launch_bounds__(256) void k_gemm_bf3(GemmArgs g0, GemmArgs g1, int KB) {
  __builtin_amdgcn_s_setprio(3);
  GemmArgs g;
  int task;
  if (!gemm_pick(g0, g1, g, task)) return;
  const GemmTask tk = g.tasks[task];
  const int ld = g.ldx, ldy = g.ldy, mode = g.mode;
  const int nrb = tk.nrb > 0 ? min(tk.nrb, g.nrb) : g.nrb;
  const int K = tk.klen > 0 ? min(tk.klen, g.klen) : g.klen;
  const int32_t *__restrict__ src = g.src;
  const int32_t *__restrict__ dst = g.dst;
  const float *__restrict__ X = (const float *)g.X;
  float *__restrict__ Y = (float *)g.Y;
  const uint4 *__restrict__ A = (const uint4 *)g.pool + (int64_t)tk.mat * g.mstride;
  __shared__ unsigned short Bh[NT][64 + 8], Bl[NT][64 + 8];
  __shared__ int32_t s_src[NT];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = (int)blockIdx.y * 4 + (tid >> 6);
  for (int i = tid; i < NT; i += 256) s_src[i] = i < tk.ncol ? src[tk.col0 + i] : -1;
  floatx4 acc[RBW][NT / 16];
#pragma unroll
  for (int r = 0; r < RBW; ++r)
#pragma unroll
    for (int cb = 0; cb < NT / 16; ++cb) acc[r][cb] = floatx4{0, 0, 0, 0};
  __syncthreads();
  const int spart = (tid & 3) * 16;
  for (int kc = 0; kc < K; kc += 64) {
#pragma unroll
    for (int sp = 0; sp < NT / 64; ++sp) {
      const int scol = sp * 64 + (tid >> 2);
      const int k0 = kc + spart;
      const int row = s_src[scol];
      float vals[16];
      if (row >= 0 && k0 < K && k0 < ld) {  // k beyond the row (padding to 32) reads as zero
        const floatx4 *p = reinterpret_cast<const floatx4 *>(X + (int64_t)row * ld + k0);
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          floatx4 v = p[q4];
          vals[q4 * 4 + 0] = v[0]; vals[q4 * 4 + 1] = v[1]; vals[q4 * 4 + 2] = v[2]; vals[q4 * 4 + 3] = v[3];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) vals[e] = 0.f;
      }
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const unsigned short h = f2bf_rne(vals[e]);
        Bh[scol][spart + e] = h;
        Bl[scol][spart + e] = f2bf_rne(vals[e] - bf2f(h));
      }
    }
    __syncthreads();
#pragma unroll
    for (int kb2 = 0; kb2 < 2; ++kb2) {
      const int gkb = (kc >> 5) + kb2;
      if (gkb * 32 < K) {
        bf16x8 ah[RBW], al[RBW];
#pragma unroll
        for (int r = 0; r < RBW; ++r) {
          const int rb = wave * RBW + r;
          if (rb < nrb) {
            const uint4 *f = A + ((int64_t)(rb * KB + gkb) * 2) * 64 + lane;
            uint4 h = f[0], l = f[64];
            ah[r] = __builtin_bit_cast(bf16x8, h);
            al[r] = __builtin_bit_cast(bf16x8, l);
          }
        }
        const int ko = kb2 * 32 + 8 * (lane >> 4);
#pragma unroll
        for (int cb = 0; cb < NT / 16; ++cb) {
          const int col = cb * 16 + (lane & 15);
          const bf16x8 bh = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&Bh[col][ko]));
          const bf16x8 bl = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(&Bl[col][ko]));
#pragma unroll
          for (int r = 0; r < RBW; ++r) {
            if (wave * RBW + r < nrb) {
              acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[r], bh, acc[r][cb], 0, 0, 0);
              acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[r], bl, acc[r][cb], 0, 0, 0);
              acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[r], bh, acc[r][cb], 0, 0, 0);
            }
          }
        }
      }
    }
    __syncthreads();
  }
  const float alpha = (float)tk.alpha;
#pragma unroll
  for (int r = 0; r < RBW; ++r) {
    const int rb = wave * RBW + r;
    if (rb >= nrb) continue;
    const int i0 = rb * 16 + 4 * (lane >> 4);
#pragma unroll
    for (int cb = 0; cb < NT / 16; ++cb) {
      const int c = cb * 16 + (lane & 15);
      if (c >= tk.ncol) continue;
      float *y = Y + (int64_t)dst[tk.col0 + c] * ldy + i0;
      const floatx4 v = acc[r][cb] * alpha;
      if (mode == GEMM_STORE) {
        *reinterpret_cast<floatx4 *>(y) = v;
      } else {
        floatx4 o = *reinterpret_cast<floatx4 *>(y);
        *reinterpret_cast<floatx4 *>(y) = o + v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Point-kernel evaluation.  KERN 0 = Laplace 1/r, 1 = Yukawa exp(-kappa r)/r.
// g and f = -(1/r) dg/dr for a pair at squared distance r2 (0 for r2 == 0).
// ---------------------------------------------------------------------------
template <typename T, int KERN>
__device__ inline void pair_gf(T r2, T kappa, T &g, T &f) {
  const T invr = r2 > (T)0 ? dev_rsqrt(r2) : (T)0;
  if (KERN == 0) {
    g = invr;
    f = invr * invr * invr;
  } else {
    const T r = r2 * invr;
    const T e = dev_exp(-kappa * r);
    g = e * invr;
    f = ((T)1 + kappa * r) * e * invr * invr * invr;
  }
}

// Fused leaf kernel.  One wave per tile of up to 64 targets of a leaf, one
// target per lane.  Sources are read with wave-uniform addresses (scalar
// loads) and broadcast to all lanes for free:
//   near point ranges (U list, small W-list boxes, direct X list): P2P
//   W-list upward equivalent surfaces: M2P
//   the leaf's own downward equivalent surface: L2P
// A tile of at most 32 (16) targets runs split into 2 (4) sub-waves that
// hold the same targets and take sources in turn (vector loads, one per
// sub-wave); the sub-wave sums are added at the end, the upper half onto the
// lower first, then (split 4) the upper quarter of what is left.  With one density column the source charge
// travels in the fourth component of the point record.  Only a range that
// contains the tile's own leaf can hold a source at zero distance, so only
// that range pays for the exclusion test (points in different leaves have
// different Morton cells; surfaces never touch the targets they serve),
// and a range counts as holding it when it overlaps the leaf's points.
// Writes potential (and gradient) times `scale` in the caller's order.
template <typename T, int KERN, bool CHECK, int NR>
__device__ __forceinline__ void leaf_pair(T xi, T yi, T zi, T sx, T sy, T sz, const T (&qv)[NR], T kappa, T kl2,
                                          T (&ap)[NR], T (&agx)[NR], T (&agy)[NR], T (&agz)[NR]) {
  const T dx = xi - sx, dy = yi - sy, dz = zi - sz;
  const T r2 = dx * dx + dy * dy + dz * dz;
  T invr = dev_rsqrt(r2);
  if (CHECK) invr = r2 > (T)0 ? invr : (T)0;
  T g, f;
  if (KERN == 0) {
    g = invr;
    f = invr * invr * invr;
  } else {
    const T r = r2 * invr;
    g = dev_exp2(-kl2 * r) * invr;
    f = g * (invr * invr + kappa * invr);  // (1 + kappa r) g / r^2
  }
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    ap[c] += g * qv[c];
    const T fq = f * qv[c];
    agx[c] -= fq * dx;
    agy[c] -= fq * dy;
    agz[c] -= fq * dz;
  }
}

template <typename T, int NR, int KERN>
__global__ __launch_bounds__(64) void k_leaf_eval(
    const int32_t *__restrict__ items, const int32_t *__restrict__ leaves, const T *__restrict__ pts,
    const T *__restrict__ qs, int64_t N, const int32_t *__restrict__ box_begin, const int32_t *__restrict__ box_end,
    const T *__restrict__ surf, int nsurf, int ld, const int32_t *__restrict__ near_off,
    const int32_t *__restrict__ near_rng, const T *__restrict__ near_o, const int32_t *__restrict__ far_off,
    const int32_t *__restrict__ far_idx, const T *__restrict__ far_o,
    const T *__restrict__ equ, const T *__restrict__ eqd, T *__restrict__ parts, const int32_t *__restrict__ perm,
    T *__restrict__ pot, T *__restrict__ grad, T kappa, T scale) {
  using V4 = typename Vec4<T>::type;
  const V4 *__restrict__ p4 = reinterpret_cast<const V4 *>(pts);
  const V4 *__restrict__ s4 = reinterpret_cast<const V4 *>(surf);
  const int item = blockIdx.x;
  const int slot = items[4 * item];
  const int code = items[4 * item + 1];
  const int part = items[4 * item + 2];
  const int split = code >> 24;
  const int b = leaves[slot];
  const int lb = box_begin[b], le = box_end[b];
  const int tb = lb + (code & 0xffffff);
  const int lane = threadIdx.x;
  const int sub = split == 1 ? 0 : lane / (64 / split);  // sub-wave
  const int tl = lane & (64 / split - 1);
  const int m = min(64 / split, le - tb);
  const bool active = tl < m;
  const V4 xv = p4[tb + (active ? tl : 0)];
  const T xi = xv[0], yi = xv[1], zi = xv[2];
  const T kl2 = kappa * (T)1.4426950408889634;  // kappa * log2(e)
  T ap[NR], agx[NR], agy[NR], agz[NR];
#pragma unroll
  for (int c = 0; c < NR; ++c) ap[c] = agx[c] = agy[c] = agz[c] = (T)0;

  // near field: point ranges
  const int u1 = near_off[item + 1];
  for (int u = near_off[item]; u < u1; ++u) {
    const int j0 = near_rng[2 * u], j1 = near_rng[2 * u + 1];
    const bool self = j0 < le && lb < j1;  // overlaps the tile's own leaf
    // targets in the source leaf's frame (one shift per range)
    const T xt = xi - near_o[4 * u], yt = yi - near_o[4 * u + 1], zt = zi - near_o[4 * u + 2];
    if (split == 1) {
      auto body = [&](int j, auto chk) {
        const V4 sp = p4[j];
        T qv[NR];
        if (NR == 1) qv[0] = sp[3];
        else {
#pragma unroll
          for (int c = 0; c < NR; ++c) qv[c] = qs[(int64_t)c * N + j];
        }
        leaf_pair<T, KERN, decltype(chk)::value, NR>(xt, yt, zt, sp[0], sp[1], sp[2], qv, kappa, kl2, ap, agx, agy, agz);
      };
      if (self) {
#pragma unroll 4
        for (int j = j0; j < j1; ++j) body(j, std::true_type());
      } else {
#pragma unroll 8
        for (int j = j0; j < j1; ++j) body(j, std::false_type());
      }
    } else {
      // split into 2 or 4 sub-waves: sub-wave h takes sources j0 + h,
      // j0 + h + split, ...; a count that is not a multiple of split leaves
      // the last steps of the upper sub-waves with a zero charge
      auto body = [&](int j, auto chk) {
        const int jj = j + sub;
        const bool ok = jj < j1;
        const V4 sp = p4[ok ? jj : j];
        T qv[NR];
        if (NR == 1) qv[0] = ok ? sp[3] : (T)0;
        else {
#pragma unroll
          for (int c = 0; c < NR; ++c) qv[c] = ok ? qs[(int64_t)c * N + jj] : (T)0;
        }
        leaf_pair<T, KERN, decltype(chk)::value, NR>(xt, yt, zt, sp[0], sp[1], sp[2], qv, kappa, kl2, ap, agx, agy, agz);
      };
      if (self) {
#pragma unroll 2
        for (int j = j0; j < j1; j += split) body(j, std::true_type());
      } else {
#pragma unroll 4
        for (int j = j0; j < j1; j += split) body(j, std::false_type());
      }
    }
  }
  // far field: W-list upward equivalent surfaces and the own downward one
  const int f1 = far_off[item + 1];
  for (int k = far_off[item]; k < f1; ++k) {
    const int fe = far_idx[k];
    const bool own = (fe >> 30) & 1;
    const int a = fe & 0x3fffffff;
    // surface centre in the target leaf's frame, and radius
    const T cx = far_o[4 * k], cy = far_o[4 * k + 1], cz = far_o[4 * k + 2], rr = far_o[4 * k + 3];
    // targets relative to the surface centre (one shift per surface; each
    // source then costs one fused multiply-add per coordinate)
    const T xt = xi - cx, yt = yi - cy, zt = zi - cz;
    const T *__restrict__ dens = (own ? eqd : equ) + (int64_t)a * NR * ld;
    if (split == 1) {
#pragma unroll 4
      for (int j = 0; j < nsurf; ++j) {
        const V4 g = s4[j];
        T qv[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) qv[c] = dens[(int64_t)c * ld + j];
        leaf_pair<T, KERN, false, NR>(xt, yt, zt, rr * g[0], rr * g[1], rr * g[2], qv, kappa, kl2, ap,
                                      agx, agy, agz);
      }
    } else {
#pragma unroll 2
      for (int j = 0; j < nsurf; j += split) {
        const int jj = j + sub;
        const bool ok = jj < nsurf;
        const V4 g = s4[ok ? jj : j];
        T qv[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) qv[c] = ok ? dens[(int64_t)c * ld + jj] : (T)0;
        leaf_pair<T, KERN, false, NR>(xt, yt, zt, rr * g[0], rr * g[1], rr * g[2], qv, kappa, kl2, ap,
                                      agx, agy, agz);
      }
    }
  }
  if (split >= 2) {
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      ap[c] += __shfl_xor(ap[c], 32);
      agx[c] += __shfl_xor(agx[c], 32);
      agy[c] += __shfl_xor(agy[c], 32);
      agz[c] += __shfl_xor(agz[c], 32);
    }
  }
  if (split == 4) {
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      ap[c] += __shfl_xor(ap[c], 16);
      agx[c] += __shfl_xor(agx[c], 16);
      agy[c] += __shfl_xor(agy[c], 16);
      agz[c] += __shfl_xor(agz[c], 16);
    }
  }
  if (part >= 0) {
    // partial sums of a split tile: [part][column][component][lane]
    if (sub == 0) {
      T *pp = parts + (int64_t)part * NR * 4 * 64;
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        pp[(c * 4 + 0) * 64 + tl] = ap[c];
        pp[(c * 4 + 1) * 64 + tl] = agx[c];
        pp[(c * 4 + 2) * 64 + tl] = agy[c];
        pp[(c * 4 + 3) * 64 + tl] = agz[c];
      }
    }
    return;
  }
  if (active && sub == 0) {
    const int64_t o = perm[tb + tl];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      pot[(int64_t)c * N + o] = ap[c] * scale;
      if (grad) {
        T *gp = grad + ((int64_t)c * N + o) * 3;
        gp[0] = agx[c] * scale;
        gp[1] = agy[c] * scale;
        gp[2] = agz[c] * scale;
      }
    }
  }
}

// Sum of the parts of split tiles, in part order; one wave per tile.
// blockIdx.y = 1 takes a second plan's parts and outputs (pair evaluation).
template <typename T, int NR>
__global__ __launch_bounds__(64) void k_leaf_parts(const int32_t *__restrict__ tiles, const int32_t *__restrict__ leaves,
                                                   const int32_t *__restrict__ box_begin,
                                                   const int32_t *__restrict__ box_end, const T *__restrict__ parts0,
                                                   const int32_t *__restrict__ perm, int64_t N, T *__restrict__ pot0,
                                                   T *__restrict__ grad0, T scale, const T *__restrict__ parts1,
                                                   T *__restrict__ pot1, T *__restrict__ grad1) {
  const bool second = blockIdx.y != 0;
  const T *__restrict__ parts = second ? parts1 : parts0;
  T *__restrict__ pot = second ? pot1 : pot0;
  T *__restrict__ grad = second ? grad1 : grad0;
  const int slot = tiles[4 * blockIdx.x], code = tiles[4 * blockIdx.x + 1];
  const int p0 = tiles[4 * blockIdx.x + 2], np = tiles[4 * blockIdx.x + 3];
  const int split = code >> 24;
  const int b = leaves[slot];
  const int tb = box_begin[b] + (code & 0xffffff);
  const int m = min(64 / split, box_end[b] - tb);
  const int lane = threadIdx.x;
  if (lane >= m) return;
  const int64_t o = perm[tb + lane];
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    T acc[4] = {0, 0, 0, 0};
    const T *pp = parts + (int64_t)p0 * NR * 4 * 64 + c * 4 * 64 + lane;
    const int64_t ps = (int64_t)NR * 4 * 64;  // one part
    // eight parts' loads in flight at a time; the sums still run in part order
    int k = 0;
    for (; k + 8 <= np; k += 8) {
      T v[8][4];
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) v[j][e] = pp[(k + j) * ps + e * 64];
#pragma unroll
      for (int j = 0; j < 8; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] += v[j][e];
    }
    for (; k < np; ++k)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] += pp[k * ps + e * 64];
    pot[(int64_t)c * N + o] = acc[0] * scale;
    if (grad) {
      T *gp = grad + ((int64_t)c * N + o) * 3;
      gp[0] = acc[1] * scale;
      gp[1] = acc[2] * scale;
      gp[2] = acc[3] * scale;
    }
  }
}

// ---------------------------------------------------------------------------
// Pair evaluation: a Laplace and a Yukawa plan on one tree (same points,
// ncrit and p).  One distance, one reciprocal square root and one set of
// source loads serve both kernels.  The leaf work is split in two launches
// over the same items: the near field (point ranges), which needs only the
// densities and so runs while the two kernels' far-field passes run on other
// streams, and the far field (W-list and own downward surfaces) after them.
// The near launch leaves every lane's running sums in `acc`
// ([item][kernel][column][pot, gx, gy, gz][lane]); the far launch continues
// them, so each sum is accumulated in the same order as by k_leaf_eval.
// ---------------------------------------------------------------------------
template <typename T, bool CHECK, int NR, bool GRAD = true>
__device__ __forceinline__ void leaf_pair_ly(T xi, T yi, T zi, T sx, T sy, T sz, const T (&qa)[NR], const T (&qb)[NR],
                                             T kappa, T kl2, T (&pa)[NR], T (&xa)[NR], T (&ya)[NR], T (&za)[NR],
                                             T (&pb)[NR], T (&xb)[NR], T (&yb)[NR], T (&zb)[NR]) {
  const T dx = xi - sx, dy = yi - sy, dz = zi - sz;
  const T r2 = dx * dx + dy * dy + dz * dz;
  T invr = dev_rsqrt(r2);
  if (CHECK) invr = r2 > (T)0 ? invr : (T)0;
  const T i2 = invr * invr;
  const T fl = i2 * invr;                       // Laplace: g = 1/r, f = 1/r^3
  const T r = r2 * invr;
  const T gy = dev_exp2(-kl2 * r) * invr;       // Yukawa: g = e^{-kappa r}/r
  const T fy = gy * (i2 + kappa * invr);        //         f = (1 + kappa r) g / r^2
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    pa[c] += invr * qa[c];
    pb[c] += gy * qb[c];
    if (GRAD) {
      const T fqa = fl * qa[c];
      xa[c] -= fqa * dx;
      ya[c] -= fqa * dy;
      za[c] -= fqa * dz;
      const T fqb = fy * qb[c];
      xb[c] -= fqb * dx;
      yb[c] -= fqb * dy;
      zb[c] -= fqb * dz;
    }
  }
}

template <typename T, int NR>
__global__ __launch_bounds__(64) void k_near_pair(
    const int32_t *__restrict__ items, const int32_t *__restrict__ leaves, const T *__restrict__ pts,
    const T *__restrict__ qs, int64_t N, const int32_t *__restrict__ box_begin, const int32_t *__restrict__ box_end,
    const int32_t *__restrict__ near_off, const int32_t *__restrict__ near_rng, const T *__restrict__ near_o,
    T *__restrict__ acc, T kappa, int nitems, int item0) {
  using V4 = typename Vec4<T>::type;
  const V4 *__restrict__ p4 = reinterpret_cast<const V4 *>(pts);
  // one wave per item (the loop also serves a grid smaller than the item
  // count: waves then take items round robin, longest first)
  // items item0 .. item0 + nitems - 1
  for (int item = item0 + (int)blockIdx.x; item < item0 + nitems; item += gridDim.x) {
    const int slot = items[4 * item];
    const int code = items[4 * item + 1];
    const int split = code >> 24;
    const int b = leaves[slot];
    const int lb = box_begin[b], le = box_end[b];
    const int tb = lb + (code & 0xffffff);
    const int lane = threadIdx.x;
    const int sub = split == 1 ? 0 : lane / (64 / split);  // sub-wave
    const int tl = lane & (64 / split - 1);
    const int m = min(64 / split, le - tb);
    const bool active = tl < m;
    const V4 xv = p4[tb + (active ? tl : 0)];
    const T xi = xv[0], yi = xv[1], zi = xv[2];
    const T kl2 = kappa * (T)1.4426950408889634;  // kappa * log2(e)
    T pa[NR], xa[NR], ya[NR], za[NR], pb[NR], xb[NR], yb[NR], zb[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) pa[c] = xa[c] = ya[c] = za[c] = pb[c] = xb[c] = yb[c] = zb[c] = (T)0;
    const int u1 = near_off[item + 1];
    for (int u = near_off[item]; u < u1; ++u) {
      const int j0 = near_rng[2 * u], j1 = near_rng[2 * u + 1];
      const bool self = j0 < le && lb < j1;
      const T xt = xi - near_o[4 * u], yt = yi - near_o[4 * u + 1], zt = zi - near_o[4 * u + 2];
      if (split == 1) {
        auto body = [&](int j, auto chk) {
          const V4 sp = p4[j];
          T qv[NR];
          if (NR == 1) qv[0] = sp[3];
          else {
#pragma unroll
            for (int c = 0; c < NR; ++c) qv[c] = qs[(int64_t)c * N + j];
          }
          leaf_pair_ly<T, decltype(chk)::value, NR>(xt, yt, zt, sp[0], sp[1], sp[2], qv, qv, kappa, kl2, pa, xa, ya,
                                                     za, pb, xb, yb, zb);
        };
        if (self) {
#pragma unroll 4
          for (int j = j0; j < j1; ++j) body(j, std::true_type());
        } else {
#pragma unroll 8
          for (int j = j0; j < j1; ++j) body(j, std::false_type());
        }
      } else {
        auto body = [&](int j, auto chk) {
          const int jj = j + sub;
          const bool ok = jj < j1;
          const V4 sp = p4[ok ? jj : j];
          T qv[NR];
          if (NR == 1) qv[0] = ok ? sp[3] : (T)0;
          else {
#pragma unroll
            for (int c = 0; c < NR; ++c) qv[c] = ok ? qs[(int64_t)c * N + jj] : (T)0;
          }
          leaf_pair_ly<T, decltype(chk)::value, NR>(xt, yt, zt, sp[0], sp[1], sp[2], qv, qv, kappa, kl2, pa, xa, ya,
                                                     za, pb, xb, yb, zb);
        };
        if (self) {
#pragma unroll 2
          for (int j = j0; j < j1; j += split) body(j, std::true_type());
        } else {
#pragma unroll 4
          for (int j = j0; j < j1; j += split) body(j, std::false_type());
        }
      }
    }
    T *a = acc + (int64_t)item * 2 * NR * 4 * 64;
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      a[(c * 4 + 0) * 64 + lane] = pa[c];
      a[(c * 4 + 1) * 64 + lane] = xa[c];
      a[(c * 4 + 2) * 64 + lane] = ya[c];
      a[(c * 4 + 3) * 64 + lane] = za[c];
      a[((NR + c) * 4 + 0) * 64 + lane] = pb[c];
      a[((NR + c) * 4 + 1) * 64 + lane] = xb[c];
      a[((NR + c) * 4 + 2) * 64 + lane] = yb[c];
      a[((NR + c) * 4 + 3) * 64 + lane] = zb[c];
    }
  }
}

template <typename T, int NR>
__device__ __forceinline__ void leaf_store(int part, int sub, bool active, int tl, int tb, T *__restrict__ parts,
                                           const int32_t *__restrict__ perm, int64_t N, T *__restrict__ pot,
                                           T *__restrict__ grad, T scale, const T (&ap)[NR], const T (&agx)[NR],
                                           const T (&agy)[NR], const T (&agz)[NR]) {
  if (part >= 0) {
    if (sub == 0) {
      T *pp = parts + (int64_t)part * NR * 4 * 64;
#pragma unroll
      for (int c = 0; c < NR; ++c) {
        pp[(c * 4 + 0) * 64 + tl] = ap[c];
        pp[(c * 4 + 1) * 64 + tl] = agx[c];
        pp[(c * 4 + 2) * 64 + tl] = agy[c];
        pp[(c * 4 + 3) * 64 + tl] = agz[c];
      }
    }
    return;
  }
  if (active && sub == 0) {
    const int64_t o = perm[tb + tl];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      pot[(int64_t)c * N + o] = ap[c] * scale;
      if (grad) {
        T *gp = grad + ((int64_t)c * N + o) * 3;
        gp[0] = agx[c] * scale;
        gp[1] = agy[c] * scale;
        gp[2] = agz[c] * scale;
      }
    }
  }
}

template <typename T, int NR, bool GRAD>
__global__ __launch_bounds__(64) void k_far_pair(
    const int32_t *__restrict__ items, const int32_t *__restrict__ leaves, const T *__restrict__ pts, int64_t N,
    const int32_t *__restrict__ box_begin, const int32_t *__restrict__ box_end, const T *__restrict__ surf,
    int nsurf, int ld, const int32_t *__restrict__ far_off, const int32_t *__restrict__ far_idx,
    const T *__restrict__ far_o, const T *__restrict__ acc, const T *__restrict__ equ_a,
    const T *__restrict__ eqd_a, const T *__restrict__ equ_b, const T *__restrict__ eqd_b, T *__restrict__ parts_a,
    T *__restrict__ parts_b, const int32_t *__restrict__ perm, T *__restrict__ pot_a, T *__restrict__ grad_a,
    T *__restrict__ pot_b, T *__restrict__ grad_b, T kappa, T scale) {
  using V4 = typename Vec4<T>::type;
  const V4 *__restrict__ p4 = reinterpret_cast<const V4 *>(pts);
  const V4 *__restrict__ s4 = reinterpret_cast<const V4 *>(surf);
  const int item = blockIdx.x;
  const int slot = items[4 * item];
  const int code = items[4 * item + 1];
  const int part = items[4 * item + 2];
  const int split = code >> 24;
  const int b = leaves[slot];
  const int lb = box_begin[b], le = box_end[b];
  const int tb = lb + (code & 0xffffff);
  const int lane = threadIdx.x;
  const int sub = split == 1 ? 0 : lane / (64 / split);  // sub-wave
  const int tl = lane & (64 / split - 1);
  const int m = min(64 / split, le - tb);
  const bool active = tl < m;
  const V4 xv = p4[tb + (active ? tl : 0)];
  const T xi = xv[0], yi = xv[1], zi = xv[2];
  const T kl2 = kappa * (T)1.4426950408889634;
  T pa[NR], xa[NR], ya[NR], za[NR], pb[NR], xb[NR], yb[NR], zb[NR];
  const T *a = acc + (int64_t)item * 2 * NR * 4 * 64;
#pragma unroll
  for (int c = 0; c < NR; ++c) {
    pa[c] = a[(c * 4 + 0) * 64 + lane];
    pb[c] = a[((NR + c) * 4 + 0) * 64 + lane];
    if (GRAD) {
      xa[c] = a[(c * 4 + 1) * 64 + lane];
      ya[c] = a[(c * 4 + 2) * 64 + lane];
      za[c] = a[(c * 4 + 3) * 64 + lane];
      xb[c] = a[((NR + c) * 4 + 1) * 64 + lane];
      yb[c] = a[((NR + c) * 4 + 2) * 64 + lane];
      zb[c] = a[((NR + c) * 4 + 3) * 64 + lane];
    } else {
      xa[c] = ya[c] = za[c] = xb[c] = yb[c] = zb[c] = (T)0;
    }
  }
  const int f1 = far_off[item + 1];
  for (int k = far_off[item]; k < f1; ++k) {
    const int fe = far_idx[k];
    const bool own = (fe >> 30) & 1;
    const int bx = fe & 0x3fffffff;
    const T cx = far_o[4 * k], cy = far_o[4 * k + 1], cz = far_o[4 * k + 2], rr = far_o[4 * k + 3];
    // In units of the surface radius rr (targets u = (x - c) / rr, sources
    // the unit grid g, kappa rr): g(rr s) = g_unit(s) / rr and the gradient
    // scales by 1 / rr^2, so each surface is summed in unit coordinates and
    // scaled once; a source then costs no multiply for its position.
    const T irr = (T)1 / rr;
    const T xt = (xi - cx) * irr, yt = (yi - cy) * irr, zt = (zi - cz) * irr;
    const T ku = kappa * rr, ku2 = kl2 * rr;
    const T *__restrict__ da = (own ? eqd_a : equ_a) + (int64_t)bx * NR * ld;
    const T *__restrict__ db = (own ? eqd_b : equ_b) + (int64_t)bx * NR * ld;
    T ua[NR], uxa[NR], uya[NR], uza[NR], ub[NR], uxb[NR], uyb[NR], uzb[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) ua[c] = uxa[c] = uya[c] = uza[c] = ub[c] = uxb[c] = uyb[c] = uzb[c] = (T)0;
    if (split == 1) {
#pragma unroll 4
      for (int j = 0; j < nsurf; ++j) {
        const V4 g = s4[j];
        T qa[NR], qb[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) { qa[c] = da[(int64_t)c * ld + j]; qb[c] = db[(int64_t)c * ld + j]; }
        leaf_pair_ly<T, false, NR, GRAD>(xt, yt, zt, g[0], g[1], g[2], qa, qb, ku, ku2,
                                   ua, uxa, uya, uza, ub, uxb, uyb, uzb);
      }
    } else {
#pragma unroll 2
      for (int j = 0; j < nsurf; j += split) {
        const int jj = j + sub;
        const bool ok = jj < nsurf;
        const V4 g = s4[ok ? jj : j];
        T qa[NR], qb[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) {
          qa[c] = ok ? da[(int64_t)c * ld + jj] : (T)0;
          qb[c] = ok ? db[(int64_t)c * ld + jj] : (T)0;
        }
        leaf_pair_ly<T, false, NR, GRAD>(xt, yt, zt, g[0], g[1], g[2], qa, qb, ku, ku2,
                                   ua, uxa, uya, uza, ub, uxb, uyb, uzb);
      }
    }
    const T irr2 = irr * irr;
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      pa[c] += ua[c] * irr;
      pb[c] += ub[c] * irr;
      if (GRAD) {
        xa[c] += uxa[c] * irr2; ya[c] += uya[c] * irr2; za[c] += uza[c] * irr2;
        xb[c] += uxb[c] * irr2; yb[c] += uyb[c] * irr2; zb[c] += uzb[c] * irr2;
      }
    }
  }
  if (split >= 2) {
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      pa[c] += __shfl_xor(pa[c], 32); xa[c] += __shfl_xor(xa[c], 32);
      ya[c] += __shfl_xor(ya[c], 32); za[c] += __shfl_xor(za[c], 32);
      pb[c] += __shfl_xor(pb[c], 32); xb[c] += __shfl_xor(xb[c], 32);
      yb[c] += __shfl_xor(yb[c], 32); zb[c] += __shfl_xor(zb[c], 32);
    }
  }
  if (split == 4) {
#pragma unroll
    for (int c = 0; c < NR; ++c) {
      pa[c] += __shfl_xor(pa[c], 16); xa[c] += __shfl_xor(xa[c], 16);
      ya[c] += __shfl_xor(ya[c], 16); za[c] += __shfl_xor(za[c], 16);
      pb[c] += __shfl_xor(pb[c], 16); xb[c] += __shfl_xor(xb[c], 16);
      yb[c] += __shfl_xor(yb[c], 16); zb[c] += __shfl_xor(zb[c], 16);
    }
  }
  leaf_store<T, NR>(part, sub, active, tl, tb, parts_a, perm, N, pot_a, grad_a, scale, pa, xa, ya, za);
  leaf_store<T, NR>(part, sub, active, tl, tb, parts_b, perm, N, pot_b, grad_b, scale, pb, xb, yb, zb);
}

// Surface kernel of a pair evaluation: the Laplace (YA) and Yukawa (YB)
// potentials at the surface points of box tbox[slot] from the same sources,
// one distance per pair.  One surface point per lane, a wave per 64 surface
// points (blockDim.x = 64 ceil(nsurf / 64) <= 512).  Every wave reads the
// sources itself with wave-uniform addresses (scalar loads, no LDS and no
// barrier), and the target point is moved into each source leaf's frame
// once per leaf.  Surfaces never hold a source point (check surfaces lie
// outside the boxes whose points they see, and X-list leaves are not
// adjacent to the boxes they feed), so no pair is at zero distance.
template <typename T, int NR>
__global__ __launch_bounds__(512) void k_surf_eval_pair(
    const int32_t *__restrict__ tbox, const int32_t *__restrict__ src_off, const int32_t *__restrict__ src_idx,
    const T *__restrict__ src_o,
    const T *__restrict__ pts, const T *__restrict__ qs, int64_t N, const int32_t *__restrict__ box_begin,
    const int32_t *__restrict__ box_end, const T *__restrict__ box_geom, const T *__restrict__ surf, int nsurf,
    int ld, T alpha, T *__restrict__ YA, T *__restrict__ YB, int mode, T kappa) {
  using V4 = typename Vec4<T>::type;
  const V4 *__restrict__ p4 = reinterpret_cast<const V4 *>(pts);
  const int slot = blockIdx.x;
  const int b = tbox[slot];
  const int tid = threadIdx.x;
  // target surface in the box's own frame; sources (leaf frames) shifted by
  // src_o (source leaf centre - box centre; none: the box itself)
  const T rr = box_geom[b * 4 + 3] * alpha;
  const int ii = tid < nsurf ? tid : 0;
  const T tx = rr * surf[ii * 4 + 0], ty = rr * surf[ii * 4 + 1], tz = rr * surf[ii * 4 + 2];
  const T kl2 = kappa * (T)1.4426950408889634;  // kappa * log2(e)
  T accA[NR], accB[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) accA[r] = accB[r] = (T)0;
  const int k1 = src_off[slot + 1];
  for (int k = src_off[slot]; k < k1; ++k) {
    const int a = src_idx[k];
    const T xt = src_o ? tx - src_o[4 * k] : tx, yt = src_o ? ty - src_o[4 * k + 1] : ty,
            zt = src_o ? tz - src_o[4 * k + 2] : tz;
    const int sb = box_begin[a], se = box_end[a];
#pragma unroll 8
    for (int j = sb; j < se; ++j) {
      const V4 sp = p4[j];
      const T dx = xt - sp[0], dy = yt - sp[1], dz = zt - sp[2];
      const T r2 = dx * dx + dy * dy + dz * dz;
      const T invr = dev_rsqrt(r2);
      const T gy = dev_exp2(-kl2 * (r2 * invr)) * invr;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const T q = qs[(int64_t)r * N + j];
        accA[r] += invr * q;
        accB[r] += gy * q;
      }
    }
  }
  if (tid < nsurf) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T *ya = YA + ((int64_t)b * NR + r) * ld + tid;
      T *yb = YB + ((int64_t)b * NR + r) * ld + tid;
      if (mode == 0) { *ya = accA[r]; *yb = accB[r]; }
      else { *ya += accA[r]; *yb += accB[r]; }
    }
  }
}

// ---------------------------------------------------------------------------
// Monopole + dipole sources (pair evaluation, potentials only).  Source j
// carries a charge and a dipole moment d_j; a kernel's potential at x is
//   sum_j [ c q_j g(x, y_j) + d_j . grad_y g(x, y_j) ],
// grad_y g = f(r) (x - y) with the f of the gradient formulas.  The charge
// arrives pre-scaled per kernel: the points' fourth slot holds c_a q_j and the
// dipole record's fourth slot c_b q_j.  Equivalent densities stay monopoles,
// so only the source side (P2M, P2L, near field) changes.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_permute_md(const T *__restrict__ q, const T *__restrict__ dip, const int32_t *__restrict__ perm,
                             int64_t N, T ca, T cb, T *__restrict__ pts, T *__restrict__ dips) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= N) return;
  const int64_t j = perm[i];
  const T qj = q[j];
  pts[i * 4 + 3] = ca * qj;
  dips[i * 4 + 0] = dip[3 * j + 0];
  dips[i * 4 + 1] = dip[3 * j + 1];
  dips[i * 4 + 2] = dip[3 * j + 2];
  dips[i * 4 + 3] = cb * qj;
}

template <typename T>
__global__ __launch_bounds__(512) void k_surf_eval_pair_md(
    const int32_t *__restrict__ tbox, const int32_t *__restrict__ src_off, const int32_t *__restrict__ src_idx,
    const T *__restrict__ src_o,
    const T *__restrict__ pts, const T *__restrict__ dips, const int32_t *__restrict__ box_begin,
    const int32_t *__restrict__ box_end, const T *__restrict__ box_geom, const T *__restrict__ surf, int nsurf,
    int ld, T alpha, T *__restrict__ YA, T *__restrict__ YB, T kappa) {
  __shared__ T sx[512], sy[512], sz[512], sqa[512], sdx[512], sdy[512], sdz[512], sqb[512];
  const int slot = blockIdx.x;
  const int b = tbox[slot];
  const int tid = threadIdx.x, nt = blockDim.x;
  // target surface in the box's own frame; sources (leaf frames) shifted by
  // src_o (source leaf centre - box centre; none: the box itself)
  const T cx = 0, cy = 0, cz = 0;
  const T rr = box_geom[b * 4 + 3] * alpha;
  const int ii = tid < nsurf ? tid : 0;
  const T tx = cx + rr * surf[ii * 4 + 0], ty = cy + rr * surf[ii * 4 + 1], tz = cz + rr * surf[ii * 4 + 2];
  T accA = 0, accB = 0;
  for (int k = src_off[slot]; k < src_off[slot + 1]; ++k) {
    const int a = src_idx[k];
    const T ox = src_o ? src_o[4 * k] : (T)0, oy = src_o ? src_o[4 * k + 1] : (T)0,
            oz = src_o ? src_o[4 * k + 2] : (T)0;
    const int sb = box_begin[a], se = box_end[a];
    for (int c0 = sb; c0 < se; c0 += nt) {
      const int j = c0 + tid;
      if (j < se) {
        sx[tid] = pts[(int64_t)j * 4 + 0] + ox;
        sy[tid] = pts[(int64_t)j * 4 + 1] + oy;
        sz[tid] = pts[(int64_t)j * 4 + 2] + oz;
        sqa[tid] = pts[(int64_t)j * 4 + 3];
        sdx[tid] = dips[(int64_t)j * 4 + 0];
        sdy[tid] = dips[(int64_t)j * 4 + 1];
        sdz[tid] = dips[(int64_t)j * 4 + 2];
        sqb[tid] = dips[(int64_t)j * 4 + 3];
      }
      __syncthreads();
      const int cnt = min(nt, se - c0);
      for (int j2 = 0; j2 < cnt; ++j2) {
        const T dx = tx - sx[j2], dy = ty - sy[j2], dz = tz - sz[j2];
        const T r2 = dx * dx + dy * dy + dz * dz;
        const T invr = r2 > (T)0 ? dev_rsqrt(r2) : (T)0;
        const T i2 = invr * invr;
        const T dd = sdx[j2] * dx + sdy[j2] * dy + sdz[j2] * dz;
        const T r = r2 * invr;
        const T gy = dev_exp(-kappa * r) * invr;
        accA += invr * sqa[j2] + (i2 * invr) * dd;
        accB += gy * sqb[j2] + (((T)1 + kappa * r) * gy * i2) * dd;
      }
      __syncthreads();
    }
  }
  if (tid < nsurf) {
    YA[(int64_t)b * ld + tid] = accA;
    YB[(int64_t)b * ld + tid] = accB;
  }
}

// Gradient (GRAD): grad_x [c q g + (d.u) f] = f d + ((d.u) h - c q f) u,
// u = x - y, h = f'(r)/r: Laplace -3/r^5, Yukawa
// -(kappa^2 r^2 + 3 kappa r + 3) e^{-kappa r}/r^5.
template <typename T, bool CHECK, bool GRAD = false>
__device__ __forceinline__ void leaf_pair_md(T xi, T yi, T zi, const typename Vec4<T>::type &sp,
                                             const typename Vec4<T>::type &sd, T kappa, T kl2, T &pa, T &pb,
                                             T *ga = nullptr, T *gb = nullptr) {
  const T dx = xi - sp[0], dy = yi - sp[1], dz = zi - sp[2];
  const T r2 = dx * dx + dy * dy + dz * dz;
  T invr = dev_rsqrt(r2);
  if (CHECK) invr = r2 > (T)0 ? invr : (T)0;
  const T i2 = invr * invr;
  const T dd = sd[0] * dx + sd[1] * dy + sd[2] * dz;
  const T r = r2 * invr;
  const T gy = dev_exp2(-kl2 * r) * invr;
  const T fl = i2 * invr;
  const T kr = kappa * r;
  const T fy = ((T)1 + kr) * gy * i2;
  pa += invr * sp[3] + fl * dd;
  pb += gy * sd[3] + fy * dd;
  if (GRAD) {
    const T hl = (T)-3 * fl * i2;
    const T hy = -(kr * kr + (T)3 * kr + (T)3) * gy * i2 * i2;
    const T tl = dd * hl - fl * sp[3], ty = dd * hy - fy * sd[3];
    ga[0] += fl * sd[0] + tl * dx;
    ga[1] += fl * sd[1] + tl * dy;
    ga[2] += fl * sd[2] + tl * dz;
    gb[0] += fy * sd[0] + ty * dx;
    gb[1] += fy * sd[1] + ty * dy;
    gb[2] += fy * sd[2] + ty * dz;
  }
}

// Near field of monopole + dipole sources, both kernels, potentials only;
// running sums to acc in the layout of k_near_pair with one column.
template <typename T, bool GRAD>
__global__ __launch_bounds__(64) void k_near_pair_md(
    const int32_t *__restrict__ items, const int32_t *__restrict__ leaves, const T *__restrict__ pts,
    const T *__restrict__ dips, const int32_t *__restrict__ box_begin, const int32_t *__restrict__ box_end,
    const int32_t *__restrict__ near_off, const int32_t *__restrict__ near_rng, const T *__restrict__ near_o,
    T *__restrict__ acc, T kappa, int nitems, int item0) {
  using V4 = typename Vec4<T>::type;
  const V4 *__restrict__ p4 = reinterpret_cast<const V4 *>(pts);
  const V4 *__restrict__ d4 = reinterpret_cast<const V4 *>(dips);
  // items item0 .. item0 + nitems - 1
  for (int item = item0 + (int)blockIdx.x; item < item0 + nitems; item += gridDim.x) {
    const int slot = items[4 * item];
    const int code = items[4 * item + 1];
    const int split = code >> 24;
    const int b = leaves[slot];
    const int lb = box_begin[b], le = box_end[b];
    const int tb = lb + (code & 0xffffff);
    const int lane = threadIdx.x;
    const int sub = split == 1 ? 0 : lane / (64 / split);  // sub-wave
    const int tl = lane & (64 / split - 1);
    const int m = min(64 / split, le - tb);
    const bool active = tl < m;
    const V4 xv = p4[tb + (active ? tl : 0)];
    const T xi = xv[0], yi = xv[1], zi = xv[2];
    const T kl2 = kappa * (T)1.4426950408889634;
    T pa = 0, pb = 0;
    T ga[3] = {0, 0, 0}, gb[3] = {0, 0, 0};
    const int u1 = near_off[item + 1];
    for (int u = near_off[item]; u < u1; ++u) {
      const int j0 = near_rng[2 * u], j1 = near_rng[2 * u + 1];
      const bool self = j0 < le && lb < j1;
      const T xt = xi - near_o[4 * u], yt = yi - near_o[4 * u + 1], zt = zi - near_o[4 * u + 2];
      if (split == 1) {
        if (self) {
#pragma unroll 4
          for (int j = j0; j < j1; ++j) leaf_pair_md<T, true, GRAD>(xt, yt, zt, p4[j], d4[j], kappa, kl2, pa, pb, ga, gb);
        } else {
#pragma unroll 8
          for (int j = j0; j < j1; ++j) leaf_pair_md<T, false, GRAD>(xt, yt, zt, p4[j], d4[j], kappa, kl2, pa, pb, ga, gb);
        }
      } else {
        // split into sub-waves: sub-wave h takes sources j0 + h, j0 + h +
        // split, ...; a missing last source counts with zero strength
        auto body = [&](int j, auto chk) {
          const int jj = j + sub;
          const bool ok = jj < j1;
          V4 sp = p4[ok ? jj : j], sd = d4[ok ? jj : j];
          if (!ok) { sp[3] = (T)0; sd = V4{0, 0, 0, 0}; }
          leaf_pair_md<T, decltype(chk)::value, GRAD>(xt, yt, zt, sp, sd, kappa, kl2, pa, pb, ga, gb);
        };
        if (self) {
#pragma unroll 2
          for (int j = j0; j < j1; j += split) body(j, std::true_type());
        } else {
#pragma unroll 4
          for (int j = j0; j < j1; j += split) body(j, std::false_type());
        }
      }
    }
    T *a = acc + (int64_t)item * 2 * 4 * 64;
    a[lane] = pa;
    a[4 * 64 + lane] = pb;
    if (GRAD) {
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        a[(1 + e) * 64 + lane] = ga[e];
        a[(5 + e) * 64 + lane] = gb[e];
      }
    }
  }
}

// Surface kernel: potential at the surface points (radius `alpha` * h) of
// box tbox[slot] from the points of the leaves src_idx[src_off[slot] ..].
// Y[(box*NR + r)*ld + i] (mode 0: store, 1: add).
template <typename T, int NR, int KERN>
__global__ __launch_bounds__(256) void k_surf_eval(
    const int32_t *__restrict__ tbox, const int32_t *__restrict__ src_off, const int32_t *__restrict__ src_idx,
    const T *__restrict__ src_o,
    const T *__restrict__ pts, const T *__restrict__ qs, int64_t N, const int32_t *__restrict__ box_begin,
    const int32_t *__restrict__ box_end, const T *__restrict__ box_geom, const T *__restrict__ surf, int nsurf,
    int ld, T alpha, T *__restrict__ Y, int mode, T kappa) {
  __shared__ T sx[256], sy[256], sz[256], sq[NR][256];
  const int slot = blockIdx.x;
  const int b = tbox[slot];
  const int tid = threadIdx.x;
  // target surface in the box's own frame; sources (leaf frames) shifted by
  // src_o (source leaf centre - box centre; none: the box itself)
  const T cx = 0, cy = 0, cz = 0;
  const T rr = box_geom[b * 4 + 3] * alpha;
  for (int i0 = 0; i0 < nsurf; i0 += 512) {
    T tx[2], ty[2], tz[2];
    T acc[2][NR];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = i0 + tid + h * 256;
      const int ii = i < nsurf ? i : 0;
      tx[h] = cx + rr * surf[ii * 4 + 0];
      ty[h] = cy + rr * surf[ii * 4 + 1];
      tz[h] = cz + rr * surf[ii * 4 + 2];
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[h][r] = (T)0;
    }
    for (int s = src_off[slot]; s < src_off[slot + 1]; ++s) {
      const int a = src_idx[s];
      const T ox = src_o ? src_o[4 * s] : (T)0, oy = src_o ? src_o[4 * s + 1] : (T)0,
              oz = src_o ? src_o[4 * s + 2] : (T)0;
      const int sb = box_begin[a], se = box_end[a];
      for (int c0 = sb; c0 < se; c0 += 256) {
        const int j = c0 + tid;
        if (j < se) {
          sx[tid] = pts[(int64_t)j * 4 + 0] + ox;
          sy[tid] = pts[(int64_t)j * 4 + 1] + oy;
          sz[tid] = pts[(int64_t)j * 4 + 2] + oz;
#pragma unroll
          for (int r = 0; r < NR; ++r) sq[r][tid] = qs[(int64_t)r * N + j];
        }
        __syncthreads();
        const int cnt = min(256, se - c0);
        for (int j2 = 0; j2 < cnt; ++j2) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const T dx = tx[h] - sx[j2], dy = ty[h] - sy[j2], dz = tz[h] - sz[j2];
            T gg, ff;
            pair_gf<T, KERN>(dx * dx + dy * dy + dz * dz, kappa, gg, ff);
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[h][r] += gg * sq[r][j2];
          }
        }
        __syncthreads();
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int i = i0 + tid + h * 256;
      if (i < nsurf) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          T *y = Y + ((int64_t)b * NR + r) * ld + i;
          if (mode == 0) *y = acc[h][r];
          else *y += acc[h][r];
        }
      }
    }
  }
}

// Densities into Morton order; with one column the density is also stored
// as the fourth component of the sorted point record (read by k_leaf_eval).
template <typename T>
__global__ void k_permute(const T *__restrict__ q, const int32_t *__restrict__ perm, int64_t N, int nr,
                          T *__restrict__ qs, T *__restrict__ pts) {
  int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= N) return;
  const int64_t j = perm[i];
  for (int r = 0; r < nr; ++r) qs[(int64_t)r * N + i] = q[(int64_t)r * N + j];
  if (nr == 1) pts[i * 4 + 3] = q[j];
}

template <typename T>
__global__ void k_fill_zero(T *__restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) y[i] = (T)0;
}

// y[box] = sum over the box's pairs (fixed order) of pairbuf[pair], first
// `rows` entries of each column; 4 entries per thread.  Rows of pairbuf have
// leading dimension ldp, rows of y leading dimension ld.
// blockIdx.y = 1 selects a second plan's (pairbuf, y, ldp, rows) on the same
// tree (pair evaluation).
// One box's sum (one wave, lane = 0..63).
template <typename T>
__device__ __forceinline__ void pair_reduce_box(int slot, int lane, const int32_t *__restrict__ tgt,
                                                const int32_t *__restrict__ off, const int32_t *__restrict__ pairs,
                                                const T *__restrict__ pairbuf, T *__restrict__ y, int nr, int ld,
                                                int ldp, int rows, const int32_t *__restrict__ brows,
                                                const T *__restrict__ add_) {
  using V4 = typename Vec4<T>::type;
  // add (may be null): a per-box array added after the sum (the M2L sums
  // take the P2L projections this way)
  const V4 *__restrict__ add = reinterpret_cast<const V4 *>(add_);
  const int b = tgt[slot];
  const int p0 = off[slot], p1 = off[slot + 1];
  const int rq = rows >> 2, lq = ld >> 2, pq = ldp >> 2;
  // rows of this box's slots that hold data (its level's rank); the rows
  // above it, up to `rows`, are set to zero
  const int bq = brows ? min(rq, brows[b] >> 2) : rq;
  const V4 *__restrict__ pb = reinterpret_cast<const V4 *>(pairbuf);
  for (int e = lane; e < nr * rq; e += 64) {
    const int r = e / rq, i = e - r * rq;
    if (i >= bq) {
      reinterpret_cast<V4 *>(y)[((int64_t)b * nr + r) * lq + i] =
          add ? add[((int64_t)b * nr + r) * lq + i] : V4{0, 0, 0, 0};
      continue;
    }
    // four independent partial sums (pairs p0 + 4k + j go to sum j) keep
    // four loads in flight; they are added in a fixed order
    V4 a0 = V4{0, 0, 0, 0}, a1 = a0, a2 = a0, a3 = a0;
    int p = p0;
    for (; p + 4 <= p1; p += 4) {
      a0 += pb[((int64_t)pairs[p] * nr + r) * pq + i];
      a1 += pb[((int64_t)pairs[p + 1] * nr + r) * pq + i];
      a2 += pb[((int64_t)pairs[p + 2] * nr + r) * pq + i];
      a3 += pb[((int64_t)pairs[p + 3] * nr + r) * pq + i];
    }
    if (p < p1) a0 += pb[((int64_t)pairs[p] * nr + r) * pq + i];
    if (p + 1 < p1) a1 += pb[((int64_t)pairs[p + 1] * nr + r) * pq + i];
    if (p + 2 < p1) a2 += pb[((int64_t)pairs[p + 2] * nr + r) * pq + i];
    V4 sum = (a0 + a1) + (a2 + a3);
    if (add) sum = sum + add[((int64_t)b * nr + r) * lq + i];
    reinterpret_cast<V4 *>(y)[((int64_t)b * nr + r) * lq + i] = sum;
  }
}

template <typename T>
__global__ __launch_bounds__(64) void k_pair_reduce(const int32_t *__restrict__ tgt, const int32_t *__restrict__ off,
                                                    const int32_t *__restrict__ pairs, const T *__restrict__ pairbuf0,
                                                    T *__restrict__ y0, int nr, int ld, int ldp0, int rows0,
                                                    const T *__restrict__ pairbuf1, T *__restrict__ y1, int ldp1,
                                                    int rows1, const int32_t *__restrict__ brows0,
                                                    const int32_t *__restrict__ brows1, const T *__restrict__ add0,
                                                    const T *__restrict__ add1) {
  __builtin_amdgcn_s_setprio(3);
  const bool second = blockIdx.y != 0;
  pair_reduce_box<T>((int)blockIdx.x, (int)threadIdx.x, tgt, off, pairs, second ? pairbuf1 : pairbuf0,
                     second ? y1 : y0, nr, ld, second ? ldp1 : ldp0, second ? rows1 : rows0,
                     second ? brows1 : brows0, second ? add1 : add0);
}

// Arguments of one plan's M2M sums at one level, for a chained launch.
template <typename T>
struct ReduceArgs {
  const int32_t *tgt, *off, *pairs;
  const T *pairbuf;
  T *y;
  int nr, ld, ldp, rows, nbox;
};

// Chained launch: tasks in dependency order (phase by phase); a workgroup
// takes the next task by an atomic ticket and, for a task of phase p > 0,
// first waits until every task of phase p - 1 has finished (ctr[p] counts
// them; thread 0 polls with a bounded number of sleeps and, past the bound,
// sets *err and goes on).  Tickets are taken in task order by workgroups
// that are already running, and a workgroup waits only on tasks with smaller
// tickets, so the chain drains whatever the number of resident workgroups.
// Results and stores of a task are made visible (release fence) before its
// phase counter is raised, and a waiting workgroup fences (acquire) before
// it reads them; data written in the launch is read with vector loads only.
template <typename T, int KCH>
__global__ __launch_bounds__(256) void k_chain(const ChainTask *__restrict__ tasks, int ntask,
                                               const GemmArgs *__restrict__ ga, const ReduceArgs<T> *__restrict__ ra,
                                               const int32_t *__restrict__ need, int32_t *ctr, int32_t *err,
                                               unsigned spin_limit) {
  __builtin_amdgcn_s_setprio(3);
  __shared__ int s_ticket;
  const int tid = threadIdx.x;
  // Control flow: the ticket goes through a scalar register, so the exit
  // test and every branch on the task are uniform, and each thread-0 block
  // is followed by a barrier before anything else, so no path from the end
  // of one task to the next skips a barrier (all threads reach every barrier
  // together; a loop whose latch could be reached around the thread-0 block
  // compiles into lanes that retry the old ticket forever).
  if (tid == 0) s_ticket = atomicAdd(&ctr[0], 1);
  __syncthreads();
  for (;;) {
    const int t = __builtin_amdgcn_readfirstlane(s_ticket);
    if (t >= ntask) break;
    const ChainTask tk = tasks[t];
    if (tk.phase > 0) {
      if (tid == 0) {
        const int want = need[tk.phase - 1];
        unsigned n = 0;
        while (__hip_atomic_load(&ctr[tk.phase], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < want) {
          __builtin_amdgcn_s_sleep(2);
          if (++n > spin_limit) {
            atomicOr(err, 1);
            break;
          }
        }
      }
      __syncthreads();
      __threadfence();
    }
    if (tk.kind == 0) {
      gemm_lat_tile<T, KCH>(ga[tk.arg], tk.idx >> 4, tk.idx & 15);
    } else {
      const ReduceArgs<T> r = ra[tk.arg];
      const int slot = tk.idx + (tid >> 6);
      if (slot < r.nbox)
        pair_reduce_box<T>(slot, tid & 63, r.tgt, r.off, r.pairs, r.pairbuf, r.y, r.nr, r.ld, r.ldp, r.rows,
                           (const int32_t *)nullptr, (const T *)nullptr);
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) {
      atomicAdd(&ctr[1 + tk.phase], 1);
      s_ticket = atomicAdd(&ctr[0], 1);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Evaluation driver
// ---------------------------------------------------------------------------
static GemmArgs gemm_args(const fmm_plan *P, const GemmBatch &bt, const void *X, void *Y) {
  GemmArgs g;
  g.tasks = bt.d_tasks;
  g.src = bt.d_src;
  g.dst = bt.d_dst;
  g.X = X;
  g.Y = Y;
  g.ntask = bt.ntask;
  g.nrb = bt.nrb;
  g.klen = bt.klen;
  g.ldx = bt.ldx ? bt.ldx : P->ld;
  g.ldy = bt.ldy ? bt.ldy : P->ld;
  g.S = bt.S;
  g.seg = bt.seg ? bt.seg : P->ld;
  g.KQ = bt.kq_stride ? bt.kq_stride : P->ld / 16;
  g.mode = bt.mode;
  g.nt = bt.nt;
  if (bt.pool == 2) {
    g.pool = P->pool_bf;
    g.mstride = (int64_t)(P->ld / 16) * P->bf_kb * 2 * 64;
  } else {
    g.pool = P->pool1;
    g.mstride = (int64_t)P->ld * P->ld;
  }
  return g;
}

template <typename T, int RBW>
static void launch_gemm_rbw(const GemmArgs &g0, const GemmArgs &g1, bool bf3, int KB, hipStream_t s) {
  const int nrb = std::max(g0.nrb, g1.ntask ? g1.nrb : 0);
  const unsigned gy = (unsigned)((nrb + 4 * RBW - 1) / (4 * RBW));
  const unsigned gx = 8u * (unsigned)((g0.ntask + 7) / 8 + (g1.ntask + 7) / 8);
  if constexpr (std::is_same<T, float>::value) {
    if (bf3) {
      if (g0.nt == 2 * GEMM_NT)
        hipLaunchKernelGGL((k_gemm_bf3<RBW, 2 * GEMM_NT>), dim3(gx, gy), dim3(256), 0, s, g0, g1, KB);
      else
        hipLaunchKernelGGL((k_gemm_bf3<RBW>), dim3(gx, gy), dim3(256), 0, s, g0, g1, KB);
      return;
    }
  }
  (void)KB;
  hipLaunchKernelGGL((k_gemm<T, RBW>), dim3(gx, gy), dim3(256), 0, s, g0, g1);
}

template <typename T>
static void launch_gemm_lat(const GemmArgs &g0, const GemmArgs &g1, int kch, hipStream_t s) {
  const int nrb = std::max(g0.nrb, g1.ntask ? g1.nrb : 0);
  const dim3 grid(8u * (unsigned)((g0.ntask + 7) / 8 + (g1.ntask + 7) / 8), (unsigned)((nrb + 3) / 4));
  if constexpr (std::is_same<T, double>::value) {
    if (kch <= 1) hipLaunchKernelGGL((k_gemm_lat<T, 1>), grid, dim3(256), 0, s, g0, g1);
    else hipLaunchKernelGGL((k_gemm_lat<T, 2>), grid, dim3(256), 0, s, g0, g1);
  } else {
    switch (kch) {
      case 1: hipLaunchKernelGGL((k_gemm_lat<T, 1>), grid, dim3(256), 0, s, g0, g1); break;
      case 2: hipLaunchKernelGGL((k_gemm_lat<T, 2>), grid, dim3(256), 0, s, g0, g1); break;
      case 3: hipLaunchKernelGGL((k_gemm_lat<T, 3>), grid, dim3(256), 0, s, g0, g1); break;
      case 4: hipLaunchKernelGGL((k_gemm_lat<T, 4>), grid, dim3(256), 0, s, g0, g1); break;
      default: hipLaunchKernelGGL((k_gemm_lat<T, 5>), grid, dim3(256), 0, s, g0, g1); break;
    }
  }
}

// One launch for batch bt of plan P and, when Q is given, the same batch
// bq of plan Q (a plan sharing P's tree and precision).
template <typename T>
static int launch_gemm2(fmm_plan *P, const GemmBatch &bt, const T *X, T *Y, fmm_plan *Q, const GemmBatch *bq,
                        const T *XQ, T *YQ, hipStream_t s) {
  GemmArgs g0 = gemm_args(P, bt, X, Y);
  GemmArgs g1 = g0;
  g1.ntask = 0;
  if (Q && bq && bq->ntask) g1 = gemm_args(Q, *bq, XQ, YQ);
  if (g0.ntask == 0 && g1.ntask == 0) return FMM_OK;
  if (g0.ntask == 0) { std::swap(g0, g1); g1.ntask = 0; }
  const bool bf3 = bt.pool == 2;
  const int nrb = std::max(g0.nrb, g1.ntask ? g1.nrb : 0);
  // launches of at most tune.gemm_lat workgroups (about one per compute
  // unit: the latency kernel holds many registers and much LDS) whose K
  // extent fits its staging (320 single, 128 double precision values)
  const int kch = (std::max(g0.klen, g1.ntask ? g1.klen : 0) + 63) / 64;
  const int64_t lat_wg = 8 * (int64_t)((g0.ntask + 7) / 8 + (g1.ntask + 7) / 8) * ((nrb + 3) / 4);
  if (!bf3 && lat_wg <= P->tune.gemm_lat && kch <= (std::is_same<T, double>::value ? 2 : 5)) {
    launch_gemm_lat<T>(g0, g1, kch, s);
    FMM_HIP_TRY(hipGetLastError());
    return FMM_OK;
  }
  // Small launches (few column tiles) split the row blocks over a second grid
  // dimension so that more workgroups share the work.  Large ones take one
  // group of up to 4 blocks per wave: 5 (19 row blocks at p = 10) holds so
  // many accumulators that the 30M-point pair step at p = 10 took 176 ms
  // against 119 with 4 and 120 with 2.
  int rbw = g0.ntask + g1.ntask >= 1024 ? std::min(4, (nrb + 3) / 4) : 1;
  if (P->tune.gemm_rbw > 0) rbw = std::min(P->tune.gemm_rbw, std::max(1, (nrb + 3) / 4));
  // FP64: at most two row blocks per wave (more y-groups, fewer registers,
  // more resident waves); measured on the FP64 pair evaluation: 2 -> 59.5,
  // 3 -> 54.7, 4 -> 44.5, 5 (the one-group default at p = 8) -> 53.5
  // Mpoints/s, 1 -> 47.0.  Single precision keeps one group of up to 8
  // (two blocks per wave cost 3% there).
  if (std::is_same<T, double>::value) rbw = std::min(rbw, 2);
  const int KB = P->bf_kb;
  switch (rbw) {
    case 1: launch_gemm_rbw<T, 1>(g0, g1, bf3, KB, s); break;
    case 2: launch_gemm_rbw<T, 2>(g0, g1, bf3, KB, s); break;
    case 3: launch_gemm_rbw<T, 3>(g0, g1, bf3, KB, s); break;
    case 4: launch_gemm_rbw<T, 4>(g0, g1, bf3, KB, s); break;
    case 5: launch_gemm_rbw<T, 5>(g0, g1, bf3, KB, s); break;
    case 6: launch_gemm_rbw<T, 6>(g0, g1, bf3, KB, s); break;
    case 7: launch_gemm_rbw<T, 7>(g0, g1, bf3, KB, s); break;
    case 8: launch_gemm_rbw<T, 8>(g0, g1, bf3, KB, s); break;
    default: set_error("expansion order too large for the GEMM kernel"); return FMM_EINVAL;
  }
  FMM_HIP_TRY(hipGetLastError());
  return FMM_OK;
}

// The same launch with one wave per (task, row block) (k_gemm_narrow), for
// single precision; double precision takes launch_gemm2.
template <typename T>
static int launch_gemm2_narrow(fmm_plan *P, const GemmBatch &bt, const T *X, T *Y, fmm_plan *Q, const GemmBatch *bq,
                               const T *XQ, T *YQ, hipStream_t s) {
  if constexpr (!std::is_same<T, float>::value) {
    return launch_gemm2<T>(P, bt, X, Y, Q, bq, XQ, YQ, s);
  }
  if (bt.pool == 2) return launch_gemm2<T>(P, bt, X, Y, Q, bq, XQ, YQ, s);
  GemmArgs g0 = gemm_args(P, bt, X, Y);
  GemmArgs g1 = g0;
  g1.ntask = 0;
  if (Q && bq && bq->ntask) g1 = gemm_args(Q, *bq, XQ, YQ);
  if (g0.ntask == 0 && g1.ntask == 0) return FMM_OK;
  if (g0.ntask == 0) { std::swap(g0, g1); g1.ntask = 0; }
  const int nrb = std::max(g0.nrb, g1.ntask ? g1.nrb : 0);
  const dim3 grid(8u * (unsigned)((g0.ntask + 7) / 8 + (g1.ntask + 7) / 8), (unsigned)nrb);
  hipLaunchKernelGGL((k_gemm_narrow<T>), grid, dim3(64), 0, s, g0, g1);
  FMM_HIP_TRY(hipGetLastError());
  return FMM_OK;
}

template <typename T>
static int launch_gemm(fmm_plan *P, const GemmBatch &bt, const T *X, T *Y, hipStream_t s) {
  return launch_gemm2<T>(P, bt, X, Y, nullptr, nullptr, nullptr, nullptr, s);
}

int ensure_lists(fmm_plan *P, int nr);   // host planner
int ensure_work(fmm_plan *P, int nr);

// Densities into Morton order (and, for one column, into the points' fourth
// slot).
template <typename T, int NR>
static int eval_permute(fmm_plan *P, const T *q, hipStream_t s) {
  const DevTree &D = P->dt;
  const int64_t N = P->n;
  hipEvent_t ev = prof_begin(P, FMM_PHASE_PERMUTE, s);
  hipLaunchKernelGGL(k_permute<T>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, q, D.perm, N, NR, (T *)P->qs,
                     (T *)D.pts);
  FMM_HIP_TRY(hipGetLastError());
  prof_end(P, FMM_PHASE_PERMUTE, ev, s);
  return FMM_OK;
}

// Far-field passes: P2M, upward pass, P2L, M2L, downward pass, ending with
// the downward equivalent densities of every box at level >= 2.
template <typename T, int NR, int KERN>
static int eval_passes(fmm_plan *P, hipStream_t s) {
  const DevTree &D = P->dt;
  const int64_t N = P->n;
  const int ld = P->ld;
  const PassLists &L = P->lists_by_nr[NR];
  T *qs = (T *)P->qs, *equ = (T *)P->equ, *chk = (T *)P->chk, *eqd = (T *)P->eqd, *chku = (T *)P->chku,
    *cu = (T *)P->cu, *yd = (T *)P->yd;
  const T kappa = (T)P->kappa;
  int rc;
  hipEvent_t ev;
  if (D.maxlevel < 2) return FMM_OK;
  // P2M: upward check potentials of the leaves at level >= 2
  ev = prof_begin(P, FMM_PHASE_P2M, s);
  if (P->p2m_count > 0)
    hipLaunchKernelGGL((k_surf_eval<T, NR, KERN>), dim3(P->p2m_count), dim3(256), 0, s, P->d_p2m_box,
                       P->d_p2m_off, P->d_p2m_box, (const T *)nullptr, (const T *)D.pts, qs, N, D.box_begin, D.box_end,
                       (const T *)D.box_geom, (const T *)P->surf, P->nsurf, ld, (T)ALPHA_UC, chku, 0, kappa);
  FMM_HIP_TRY(hipGetLastError());
  prof_end(P, FMM_PHASE_P2M, ev, s);
  // upward pass in singular coordinates: every leaf's U^T projection,
  // then M2M slots and per-parent sums, deepest level first
  ev = prof_begin(P, FMM_PHASE_UC2E, s);
  if ((rc = launch_gemm<T>(P, L.ut_u_all, chku, cu, s))) return rc;
  prof_end(P, FMM_PHASE_UC2E, ev, s);
  for (int l = D.maxlevel - 1; l >= 2; --l) {
    if (!L.m2m[l].ntask) continue;
    ev = prof_begin(P, FMM_PHASE_M2M, s);
    if ((rc = launch_gemm<T>(P, L.m2m[l], cu, (T *)P->mslot, s))) return rc;
    hipLaunchKernelGGL(k_pair_reduce<T>, dim3(D.m2m_n[l]), dim3(64), 0, s, D.m2m_tgt[l], D.m2m_off[l], D.m2m_kid[l],
                       (const T *)P->mslot, cu, NR, ld, ld, L.m2m[l].nrb * 16, (const T *)nullptr, (T *)nullptr, 0, 0,
                       (const int32_t *)nullptr, (const int32_t *)nullptr, (const T *)nullptr, (const T *)nullptr);
    FMM_HIP_TRY(hipGetLastError());
    prof_end(P, FMM_PHASE_M2M, ev, s);
  }
  ev = prof_begin(P, FMM_PHASE_UC2E, s);
  if ((rc = launch_gemm<T>(P, L.vs_u, cu, equ, s))) return rc;
  prof_end(P, FMM_PHASE_UC2E, ev, s);
  // P2L: X-list sources on the downward check surfaces
  ev = prof_begin(P, FMM_PHASE_P2L, s);
  if (D.nxbox > 0)
    hipLaunchKernelGGL((k_surf_eval<T, NR, KERN>), dim3(D.nxbox), dim3(256), 0, s, D.x_box, D.x_off, D.x_idx,
                       (const T *)D.x_o, (const T *)D.pts, qs, N, D.box_begin, D.box_end, (const T *)D.box_geom,
                       (const T *)P->surf, P->nsurf, ld, (T)ALPHA_DC, chk, 0, kappa);
  FMM_HIP_TRY(hipGetLastError());
  prof_end(P, FMM_PHASE_P2L, ev, s);
  // the P2L checks' projections go to their own array, added by the M2L sums
  ev = prof_begin(P, FMM_PHASE_DC2E, s);
  if ((rc = launch_gemm<T>(P, L.ut_dx, chk, (T *)P->ydx, s))) return rc;
  prof_end(P, FMM_PHASE_DC2E, ev, s);
  // M2L between singular coordinates into pair slots (rows of the largest
  // downward rank, not of the surface size), then a fixed-order sum per
  // target box (every box at level >= 2)
  ev = prof_begin(P, FMM_PHASE_M2L, s);
  if (L.m2l_r.ntask) {  // factored: R then L through the per-pair intermediate
    if ((rc = launch_gemm<T>(P, L.m2l_r, cu, (T *)P->m2l_t, s))) return rc;
    if ((rc = launch_gemm<T>(P, L.m2l, (const T *)P->m2l_t, (T *)P->pairbuf, s))) return rc;
  } else if ((rc = launch_gemm<T>(P, L.m2l, cu, (T *)P->pairbuf, s))) {
    return rc;
  }
  prof_end(P, FMM_PHASE_M2L, ev, s);
  ev = prof_begin(P, FMM_PHASE_M2L_SUM, s);
  if (D.nvbox > 0)
    hipLaunchKernelGGL(k_pair_reduce<T>, dim3(D.nvbox), dim3(64), 0, s, D.v_tgt, D.v_off, D.v_pair,
                       (const T *)P->pairbuf, yd, NR, ld, L.m2l.ldy, L.m2l.nrb * 16, (const T *)nullptr, (T *)nullptr,
                       0, 0, (const int32_t *)P->d_m2l_rows, (const int32_t *)nullptr, (const T *)P->ydx,
                       (const T *)nullptr);
  FMM_HIP_TRY(hipGetLastError());
  prof_end(P, FMM_PHASE_M2L_SUM, ev, s);
  // downward pass: L2L between singular coordinates, coarsest level first
  for (int l = 3; l <= D.maxlevel; ++l) {
    if (L.l2l[l].ntask) {
      ev = prof_begin(P, FMM_PHASE_L2L, s);
      if ((rc = launch_gemm<T>(P, L.l2l[l], yd, yd, s))) return rc;
      prof_end(P, FMM_PHASE_L2L, ev, s);
    }
  }
  ev = prof_begin(P, FMM_PHASE_DC2E, s);
  if ((rc = launch_gemm<T>(P, L.vs_d, yd, eqd, s))) return rc;
  prof_end(P, FMM_PHASE_DC2E, ev, s);
  return FMM_OK;
}

// P2L of a Laplace plan A and a Yukawa plan B on one tree: the X-list
// sources on both kernels' downward check surfaces, one launch.
template <typename T, int NR>
static int pair_p2l(fmm_plan *A, fmm_plan *B, hipStream_t s, const T *dips) {
  const DevTree &D = A->dt;
  if (D.maxlevel < 2 || D.nxbox == 0) return FMM_OK;
  const unsigned sthreads = (unsigned)(64 * ((A->nsurf + 63) / 64));
  const T kappa = (T)B->kappa;
  hipEvent_t ev = prof_begin(A, FMM_PHASE_P2L, s);
  if (dips)
    hipLaunchKernelGGL((k_surf_eval_pair_md<T>), dim3(D.nxbox), dim3(sthreads), 0, s, D.x_box, D.x_off, D.x_idx,
                       (const T *)D.x_o, (const T *)D.pts, dips, D.box_begin, D.box_end, (const T *)D.box_geom,
                       (const T *)A->surf, A->nsurf, A->ld, (T)ALPHA_DC, (T *)A->chk, (T *)B->chk, kappa);
  else
    hipLaunchKernelGGL((k_surf_eval_pair<T, NR>), dim3(D.nxbox), dim3(sthreads), 0, s, D.x_box, D.x_off, D.x_idx,
                       (const T *)D.x_o, (const T *)D.pts, (const T *)A->qs, A->n, D.box_begin, D.box_end,
                       (const T *)D.box_geom, (const T *)A->surf, A->nsurf, A->ld, (T)ALPHA_DC, (T *)A->chk,
                       (T *)B->chk, 0, kappa);
  FMM_HIP_TRY(hipGetLastError());
  prof_end(A, FMM_PHASE_P2L, ev, s);
  return FMM_OK;
}

// The far-field passes of a Laplace plan A and a Yukawa plan B on one tree,
// every pass one launch for both (densities from A's permuted copy).  The
// surface-evaluation pass P2M (VALU work) comes first and `surf_done` is
// recorded after it; the GEMM passes follow.  P2L runs on the caller's
// stream (pair_off_chain).
// Chained launches of a pair evaluation (tunable gemm_chain): the M2M
// levels of both plans (GEMM into the child slots, then the sums per parent,
// level by level) in one k_chain launch, and the L2L levels in another.
constexpr unsigned CHAIN_SPIN_LIMIT = 1u << 18;  // polls (a memory round trip and ~128 cycles each)

template <typename T, int NR>
static int build_chain(fmm_plan *A, fmm_plan *B, bool up, Chain &C) {
  const PassLists &LA = A->lists_by_nr[NR], &LB = B->lists_by_nr[NR];
  const DevTree &D = A->dt;
  std::vector<ChainTask> tasks;
  std::vector<GemmArgs> ga;
  std::vector<ReduceArgs<T>> ra;
  std::vector<int32_t> need;
  const int kmax = std::is_same<T, double>::value ? 2 : 5;
  int kch = 1, phase = 0;
  bool fits = true;
  auto add_gemm = [&](fmm_plan *P, const GemmBatch &bt, const void *X, void *Y) {
    if (!bt.ntask) return;
    const GemmArgs g = gemm_args(P, bt, X, Y);
    const int kc = (g.klen + 63) / 64;
    if (kc > kmax || bt.pool == 2 || g.nrb > 64) fits = false;
    kch = std::max(kch, kc);
    const int id = (int)ga.size();
    ga.push_back(g);
    const int gy = (g.nrb + 3) / 4;
    for (int t = 0; t < g.ntask; ++t)
      for (int y = 0; y < gy; ++y) tasks.push_back({0, phase, id, t * 16 + y});
  };
  auto end_phase = [&]() {
    int n = 0;
    for (const ChainTask &t : tasks) n += t.phase == phase;
    if (n == 0) return;
    need.push_back(n);
    ++phase;
  };
  if (up) {
    for (int l = D.maxlevel - 1; l >= 2; --l) {
      if (!LA.m2m[l].ntask) continue;
      add_gemm(A, LA.m2m[l], A->cu, A->mslot);
      add_gemm(B, LB.m2m[l], B->cu, B->mslot);
      end_phase();
      const fmm_plan *PP[2] = {A, B};
      const PassLists *LL[2] = {&LA, &LB};
      for (int k = 0; k < 2; ++k) {
        const int id = (int)ra.size();
        ra.push_back({D.m2m_tgt[l], D.m2m_off[l], D.m2m_kid[l], (const T *)PP[k]->mslot, (T *)PP[k]->cu, NR, A->ld,
                      A->ld, LL[k]->m2m[l].nrb * 16, D.m2m_n[l]});
        for (int b = 0; b < D.m2m_n[l]; b += 4) tasks.push_back({1, phase, id, b});
      }
      end_phase();
    }
  } else {
    for (int l = 3; l <= D.maxlevel; ++l) {
      if (!LA.l2l[l].ntask) continue;
      add_gemm(A, LA.l2l[l], A->yd, A->yd);
      add_gemm(B, LB.l2l[l], B->yd, B->yd);
      end_phase();
    }
  }
  C = Chain();
  if (!fits || tasks.empty()) return FMM_OK;  // ntask = 0: the per-level launches
  int rc;
  if ((rc = plan_upload(A, &C.tasks, tasks.data(), tasks.size() * sizeof(ChainTask)))) return rc;
  if ((rc = plan_upload(A, &C.gargs, ga.data(), std::max<size_t>(1, ga.size()) * sizeof(GemmArgs)))) return rc;
  if ((rc = plan_upload(A, &C.rargs, ra.data(), std::max<size_t>(1, ra.size()) * sizeof(ReduceArgs<T>)))) return rc;
  if ((rc = plan_upload(A, &C.need, need.data(), std::max<size_t>(1, need.size()) * sizeof(int32_t)))) return rc;
  C.ntask = (int)tasks.size();
  C.nphase = phase;
  C.kch = kch;
  return FMM_OK;
}

// Both chains current for (A, B, NR) and a counter array for them (ticket
// and phase counters of each chain, then the error flag).
template <typename T, int NR>
static int ensure_chains(fmm_plan *A, fmm_plan *B) {
  const std::vector<const void *> key = {B, (const void *)(intptr_t)NR, A->cu, A->mslot, A->yd, B->cu, B->mslot, B->yd};
  int rc;
  if (A->chain_up.key != key) {
    if ((rc = build_chain<T, NR>(A, B, true, A->chain_up))) return rc;
    if ((rc = build_chain<T, NR>(A, B, false, A->chain_down))) return rc;
    A->chain_up.key = A->chain_down.key = key;
  }
  const int n = 2 + A->chain_up.nphase + A->chain_down.nphase + 1;
  if (A->chain_ctr_n < n) {
    std::vector<int32_t> z(n, 0);
    if ((rc = plan_upload(A, (void **)&A->chain_ctr, z.data(), z.size() * sizeof(int32_t)))) return rc;
    A->chain_ctr_n = n;
  }
  return FMM_OK;
}

template <typename T>
static int launch_chain(const Chain &C, int32_t *ctr, int32_t *err, hipStream_t s) {
  const unsigned grid = (unsigned)std::min(C.ntask, 1024);
  const ChainTask *t = (const ChainTask *)C.tasks;
  const GemmArgs *g = (const GemmArgs *)C.gargs;
  const ReduceArgs<T> *r = (const ReduceArgs<T> *)C.rargs;
  const int32_t *nd = (const int32_t *)C.need;
  if constexpr (std::is_same<T, double>::value) {
    if (C.kch <= 1) hipLaunchKernelGGL((k_chain<T, 1>), dim3(grid), dim3(256), 0, s, t, C.ntask, g, r, nd, ctr, err, CHAIN_SPIN_LIMIT);
    else hipLaunchKernelGGL((k_chain<T, 2>), dim3(grid), dim3(256), 0, s, t, C.ntask, g, r, nd, ctr, err, CHAIN_SPIN_LIMIT);
  } else {
    switch (C.kch) {
      case 1: hipLaunchKernelGGL((k_chain<T, 1>), dim3(grid), dim3(256), 0, s, t, C.ntask, g, r, nd, ctr, err, CHAIN_SPIN_LIMIT); break;
      case 2: hipLaunchKernelGGL((k_chain<T, 2>), dim3(grid), dim3(256), 0, s, t, C.ntask, g, r, nd, ctr, err, CHAIN_SPIN_LIMIT); break;
      case 3: hipLaunchKernelGGL((k_chain<T, 3>), dim3(grid), dim3(256), 0, s, t, C.ntask, g, r, nd, ctr, err, CHAIN_SPIN_LIMIT); break;
      case 4: hipLaunchKernelGGL((k_chain<T, 4>), dim3(grid), dim3(256), 0, s, t, C.ntask, g, r, nd, ctr, err, CHAIN_SPIN_LIMIT); break;
      default: hipLaunchKernelGGL((k_chain<T, 5>), dim3(grid), dim3(256), 0, s, t, C.ntask, g, r, nd, ctr, err, CHAIN_SPIN_LIMIT); break;
    }
  }
  FMM_HIP_TRY(hipGetLastError());
  return FMM_OK;
}

template <typename T, int NR>
static int eval_passes_pair(fmm_plan *A, fmm_plan *B, hipStream_t s, int part, hipEvent_t surf_done,
                            hipEvent_t up_done, const T *dips = nullptr, bool split_m2l = false,
                            hipStream_t s3 = nullptr) {
  const DevTree &D = A->dt;
  const int64_t N = A->n;
  const int ld = A->ld;
  const PassLists &LA = A->lists_by_nr[NR], &LB = B->lists_by_nr[NR];
  const T *qs = (const T *)A->qs;
  auto W = [](void *p) { return (T *)p; };
  const T kappa = (T)B->kappa;
  int rc;
  hipEvent_t ev;
  if (D.maxlevel < 2) return FMM_OK;
  // chained M2M and L2L launches (built for this pair and column count)
  const bool chain = A->tune.gemm_chain && A->chain_ctr && !A->chain_up.key.empty() && A->chain_up.key[0] == B &&
                     A->chain_up.key[1] == (const void *)(intptr_t)NR;
  int32_t *ctr_up = A->chain_ctr, *ctr_down = A->chain_ctr + 1 + A->chain_up.nphase,
          *chain_err = A->chain_ctr + A->chain_ctr_n - 1;
  if (part == 2) goto down;
  {
  // m2l_early: the M2L of the levels >= ls runs on s3 once the M2M into
  // level ls is done (the upward coordinates of every box at those levels
  // are then final), beside the coarser M2M levels; the coarser levels' M2L
  // follows on s, which then waits for s3.  M2L tasks ascend by level.
  const bool fact = LA.m2l_r.ntask > 0 || LB.m2l_r.ntask > 0;
  const int ls = D.maxlevel - 1;
  // (s3 may be the null stream: split_m2l, not s3, says whether to split)
  const bool m2l_early = split_m2l && A->tune.m2l_early && !chain && !fact && ls >= 2 &&
                         LA.m2l_t0.size() == (size_t)D.maxlevel + 2 && LB.m2l_t0.size() == (size_t)D.maxlevel + 2;
  auto m2l_levels = [&](int l0, int l1, hipStream_t st) -> int {  // the M2L of levels [l0, l1)
    GemmBatch a = LA.m2l, b = LB.m2l;
    a.d_tasks += LA.m2l_t0[l0];
    a.ntask = LA.m2l_t0[l1] - LA.m2l_t0[l0];
    b.d_tasks += LB.m2l_t0[l0];
    b.ntask = LB.m2l_t0[l1] - LB.m2l_t0[l0];
    return launch_gemm2<T>(A, a, W(A->cu), W(A->pairbuf), B, &b, W(B->cu), W(B->pairbuf), st);
  };
  if (chain) {
    hipLaunchKernelGGL(k_fill_zero<int32_t>, dim3(1), dim3(256), 0, s, A->chain_ctr, (int64_t)A->chain_ctr_n - 1);
    FMM_HIP_TRY(hipGetLastError());
  }
  const unsigned sthreads = (unsigned)(64 * ((A->nsurf + 63) / 64));
  ev = prof_begin(A, FMM_PHASE_P2M, s);
  if (A->p2m_count > 0 && dips)
    hipLaunchKernelGGL((k_surf_eval_pair_md<T>), dim3(A->p2m_count), dim3(sthreads), 0, s, A->d_p2m_box,
                       A->d_p2m_off, A->d_p2m_box, (const T *)nullptr, (const T *)D.pts, dips, D.box_begin, D.box_end,
                       (const T *)D.box_geom, (const T *)A->surf, A->nsurf, ld, (T)ALPHA_UC, W(A->chku), W(B->chku),
                       kappa);
  else if (A->p2m_count > 0)
    hipLaunchKernelGGL((k_surf_eval_pair<T, NR>), dim3(A->p2m_count), dim3(sthreads), 0, s, A->d_p2m_box,
                       A->d_p2m_off, A->d_p2m_box, (const T *)nullptr, (const T *)D.pts, qs, N, D.box_begin, D.box_end,
                       (const T *)D.box_geom, (const T *)A->surf, A->nsurf, ld, (T)ALPHA_UC, W(A->chku), W(B->chku), 0,
                       kappa);
  FMM_HIP_TRY(hipGetLastError());
  prof_end(A, FMM_PHASE_P2M, ev, s);
  if (surf_done) FMM_HIP_TRY(hipEventRecord(surf_done, s));
  ev = prof_begin(A, FMM_PHASE_UC2E, s);
  if ((rc = launch_gemm2<T>(A, LA.ut_u_all, W(A->chku), W(A->cu), B, &LB.ut_u_all, W(B->chku), W(B->cu), s)))
    return rc;
  prof_end(A, FMM_PHASE_UC2E, ev, s);
  if (chain && A->chain_up.ntask) {
    ev = prof_begin(A, FMM_PHASE_M2M, s);
    if ((rc = launch_chain<T>(A->chain_up, ctr_up, chain_err, s))) return rc;
    prof_end(A, FMM_PHASE_M2M, ev, s);
  }
  for (int l = D.maxlevel - 1; l >= 2 && !(chain && A->chain_up.ntask); --l) {
    if (LA.m2m[l].ntask) {
      ev = prof_begin(A, FMM_PHASE_M2M, s);
      if ((rc = launch_gemm2<T>(A, LA.m2m[l], W(A->cu), W(A->mslot), B, &LB.m2m[l], W(B->cu), W(B->mslot), s)))
        return rc;
      hipLaunchKernelGGL(k_pair_reduce<T>, dim3(D.m2m_n[l], 2), dim3(64), 0, s, D.m2m_tgt[l], D.m2m_off[l],
                         D.m2m_kid[l], (const T *)A->mslot, W(A->cu), NR, ld, ld, LA.m2m[l].nrb * 16,
                         (const T *)B->mslot, W(B->cu), ld, LB.m2m[l].nrb * 16, (const int32_t *)nullptr,
                         (const int32_t *)nullptr, (const T *)nullptr, (const T *)nullptr);
      FMM_HIP_TRY(hipGetLastError());
      prof_end(A, FMM_PHASE_M2M, ev, s);
    }
    if (m2l_early && l == ls) {
      FMM_HIP_TRY(hipEventRecord(A->ev_m2m, s));
      FMM_HIP_TRY(hipStreamWaitEvent(s3, A->ev_m2m, 0));
      ev = prof_begin(A, FMM_PHASE_M2L, s3);
      if ((rc = m2l_levels(ls, D.maxlevel + 1, s3))) return rc;
      prof_end(A, FMM_PHASE_M2L, ev, s3);
      FMM_HIP_TRY(hipEventRecord(A->ev_m2lf, s3));
    }
  }
  if (up_done) FMM_HIP_TRY(hipEventRecord(up_done, s));
  ev = prof_begin(A, FMM_PHASE_M2L, s);
  if (m2l_early) {
    if ((rc = m2l_levels(0, ls, s))) return rc;
    prof_end(A, FMM_PHASE_M2L, ev, s);
    FMM_HIP_TRY(hipStreamWaitEvent(s, A->ev_m2lf, 0));
  } else {
    // a factored plan first maps its upward coordinates through R (one
    // launch for the factored plans), then every plan's L (or dense operator)
    // writes the pair slots
    const bool fa = LA.m2l_r.ntask > 0, fb = LB.m2l_r.ntask > 0;
    rc = FMM_OK;
    if (fa) rc = launch_gemm2<T>(A, LA.m2l_r, W(A->cu), W(A->m2l_t), fb ? B : nullptr, &LB.m2l_r, W(B->cu), W(B->m2l_t), s);
    else if (fb) rc = launch_gemm<T>(B, LB.m2l_r, W(B->cu), W(B->m2l_t), s);
    if (rc) return rc;
    if ((rc = launch_gemm2<T>(A, LA.m2l, fa ? W(A->m2l_t) : W(A->cu), W(A->pairbuf), B, &LB.m2l,
                              fb ? W(B->m2l_t) : W(B->cu), W(B->pairbuf), s)))
      return rc;
    prof_end(A, FMM_PHASE_M2L, ev, s);
  }
  }
  if (part == 1) return FMM_OK;
down:
  // the M2L sums add the P2L projections (`ydx`, computed on another stream
  // by pair_p2l_projection and waited for by the caller)
  ev = prof_begin(A, FMM_PHASE_M2L_SUM, s);
  if (D.nvbox > 0)
    hipLaunchKernelGGL(k_pair_reduce<T>, dim3(D.nvbox, 2), dim3(64), 0, s, D.v_tgt, D.v_off, D.v_pair,
                       (const T *)A->pairbuf, W(A->yd), NR, ld, LA.m2l.ldy, LA.m2l.nrb * 16, (const T *)B->pairbuf,
                       W(B->yd), LB.m2l.ldy, LB.m2l.nrb * 16, (const int32_t *)A->d_m2l_rows,
                       (const int32_t *)B->d_m2l_rows, (const T *)A->ydx, (const T *)B->ydx);
  FMM_HIP_TRY(hipGetLastError());
  prof_end(A, FMM_PHASE_M2L_SUM, ev, s);
  if (chain && A->chain_down.ntask) {
    ev = prof_begin(A, FMM_PHASE_L2L, s);
    if ((rc = launch_chain<T>(A->chain_down, ctr_down, chain_err, s))) return rc;
    prof_end(A, FMM_PHASE_L2L, ev, s);
  }
  // with gemm_narrow the downward passes use one-wave workgroups, which
  // find room beside the near field's waves (pass orders 3 and 4 run them there)
  for (int l = 3; l <= D.maxlevel && !(chain && A->chain_down.ntask); ++l) {
    if (!LA.l2l[l].ntask) continue;
    ev = prof_begin(A, FMM_PHASE_L2L, s);
    rc = A->tune.gemm_narrow
             ? launch_gemm2_narrow<T>(A, LA.l2l[l], W(A->yd), W(A->yd), B, &LB.l2l[l], W(B->yd), W(B->yd), s)
             : launch_gemm2<T>(A, LA.l2l[l], W(A->yd), W(A->yd), B, &LB.l2l[l], W(B->yd), W(B->yd), s);
    if (rc) return rc;
    prof_end(A, FMM_PHASE_L2L, ev, s);
  }
  ev = prof_begin(A, FMM_PHASE_DC2E, s);
  rc = A->tune.gemm_narrow
           ? launch_gemm2_narrow<T>(A, LA.vs_d, W(A->yd), W(A->eqd), B, &LB.vs_d, W(B->yd), W(B->eqd), s)
           : launch_gemm2<T>(A, LA.vs_d, W(A->yd), W(A->eqd), B, &LB.vs_d, W(B->yd), W(B->eqd), s);
  if (rc) return rc;
  prof_end(A, FMM_PHASE_DC2E, ev, s);
  return FMM_OK;
}

template <typename T, int NR, int KERN>
static int eval_chunk(fmm_plan *P, const T *q, T *pot, T *grad, hipStream_t s) {
  const DevTree &D = P->dt;
  const int64_t N = P->n;
  const int ld = P->ld;
  T *qs = (T *)P->qs, *equ = (T *)P->equ, *eqd = (T *)P->eqd;
  const T kappa = (T)P->kappa;
  int rc;
  if ((rc = eval_permute<T, NR>(P, q, s))) return rc;
  if ((rc = eval_passes<T, NR, KERN>(P, s))) return rc;
  const T scale = (T)(1.0 / (4.0 * M_PI));
  hipEvent_t ev = prof_begin(P, FMM_PHASE_LEAF, s);
  if (D.nitems > 0)
    hipLaunchKernelGGL((k_leaf_eval<T, NR, KERN>), dim3(D.nitems), dim3(64), 0, s, D.items, D.leaves,
                       (const T *)D.pts, qs, N, D.box_begin, D.box_end, (const T *)P->surf, P->nsurf, ld,
                       D.near_off, D.near_rng, (const T *)D.near_o, D.far_off, D.far_idx, (const T *)D.far_o, equ,
                       eqd, (T *)D.parts, D.perm, pot, grad, kappa, scale);
  if (D.nsplit > 0)
    hipLaunchKernelGGL((k_leaf_parts<T, NR>), dim3(D.nsplit, 1), dim3(64), 0, s, D.split_tiles, D.leaves,
                       D.box_begin, D.box_end, (const T *)D.parts, D.perm, N, pot, grad, scale, (const T *)nullptr,
                       (T *)nullptr, (T *)nullptr);
  FMM_HIP_TRY(hipGetLastError());
  prof_end(P, FMM_PHASE_LEAF, ev, s);
  return FMM_OK;
}

template <typename T, int KERN>
static int eval_nr(fmm_plan *P, int nr, const T *q, T *pot, T *grad, hipStream_t s) {
  switch (nr) {
    case 1: return eval_chunk<T, 1, KERN>(P, q, pot, grad, s);
    case 2: return eval_chunk<T, 2, KERN>(P, q, pot, grad, s);
    case 3: return eval_chunk<T, 3, KERN>(P, q, pot, grad, s);
    case 4: return eval_chunk<T, 4, KERN>(P, q, pot, grad, s);
  }
  set_error("bad column count");
  return FMM_EINVAL;
}

template <typename T>
static int eval_typed(fmm_plan *P, const T *q, int nrhs, T *pot, T *grad, hipStream_t s) {
  const int64_t N = P->n;
  for (int c0 = 0; c0 < nrhs; c0 += MAX_NR) {
    const int nr = std::min(MAX_NR, nrhs - c0);
    int rc;
    if ((rc = ensure_work(P, nr))) return rc;
    if ((rc = ensure_lists(P, nr))) return rc;
    const T *qc = q + (int64_t)c0 * N;
    T *pc = pot + (int64_t)c0 * N;
    T *gc = grad ? grad + (int64_t)c0 * N * 3 : nullptr;
    rc = (P->kernel == FMM_YUKAWA) ? eval_nr<T, 1>(P, nr, qc, pc, gc, s) : eval_nr<T, 0>(P, nr, qc, pc, gc, s);
    if (rc) return rc;
  }
  return FMM_OK;
}

int ensure_pair(fmm_plan *A, fmm_plan *B, int nr);  // host: side streams, events, near sums


// Pair evaluation of a Laplace plan A and a Yukawa plan B on one tree, every
// launch serving both kernels:
//   stream s:   permute |          | near field           | wait | far field, part sums
//   A's side:           | P2M, P2L | GEMM passes (M2M ... L2L, DC2E)  |
// (B's fork event marks the end of the surface passes.)  Measured on the
// 393k-point workload: 1.64 ms per pair against 1.70 ms with no overlap and
// 1.66 ms with the near field started at once.
// The P2L checks' projections of both plans into their own arrays (the M2L
// sums on the side stream add them), and, once the upward pass is done, the
// M2P sources' equivalent densities (only the far field reads them): on
// stream s after the near field, off the side stream's chain, which bounds
// the step.
// P2L and the projection of its check potentials (added by the M2L sums);
// B's join event marks their end.
template <typename T, int NR>
static int pair_p2l_proj(fmm_plan *A, fmm_plan *B, hipStream_t s, const T *dips) {
  const PassLists &LA = A->lists_by_nr[NR], &LB = B->lists_by_nr[NR];
  int rc = pair_p2l<T, NR>(A, B, s, dips);
  if (rc) return rc;
  hipEvent_t ev = prof_begin(A, FMM_PHASE_DC2E, s);
  rc = launch_gemm2<T>(A, LA.ut_dx, (const T *)A->chk, (T *)A->ydx, B, &LB.ut_dx, (const T *)B->chk, (T *)B->ydx, s);
  if (rc) return rc;
  prof_end(A, FMM_PHASE_DC2E, ev, s);
  FMM_HIP_TRY(hipEventRecord(B->ev_join, s));
  return FMM_OK;
}

template <typename T, int NR>
static int pair_off_chain(fmm_plan *A, fmm_plan *B, hipStream_t s, const T *dips, bool p2l, bool vsu = true) {
  const PassLists &LA = A->lists_by_nr[NR], &LB = B->lists_by_nr[NR];
  int rc;
  if (p2l && (rc = pair_p2l_proj<T, NR>(A, B, s, dips))) return rc;
  if (!vsu) return FMM_OK;
  FMM_HIP_TRY(hipStreamWaitEvent(s, A->ev_up, 0));
  hipEvent_t ev;
  ev = prof_begin(A, FMM_PHASE_UC2E, s);
  if ((rc = launch_gemm2<T>(A, LA.vs_u, (const T *)A->cu, (T *)A->equ, B, &LB.vs_u, (const T *)B->cu, (T *)B->equ, s)))
    return rc;
  prof_end(A, FMM_PHASE_UC2E, ev, s);
  return FMM_OK;
}

// Fork and join of a pair evaluation around the near-field launch `near`,
// with pass order 3 (order 4, the default, swaps the streams of the two
// chains, see below; orders 0-2 move P2L and the main near field earlier):
//   side:    P2M | UT, M2M levels, M2L | wait P2L proj. | M2L sums, L2L, DC2E
//   side2:   wait P2M (or the fork) | the early near items (near_early)
//   side3:   wait the first M2M level | the finest levels' M2L (m2l_early)
//   s:       wait P2M | P2L, its projection, M2P sources | wait M2L | main
//            near items | wait side, side2 | far field (by the caller)
// The VALU passes (P2M, P2L, near field) share the GPU with the GEMM passes,
// which are bound by memory latency rather than by issue.
template <typename T, int NR, typename Near>
static int pair_fork_join(fmm_plan *A, fmm_plan *B, hipStream_t s, const T *dips, Near near) {
  int rc;
  const bool far = A->dt.maxlevel >= 2;
  // FMM_PROFILE_SERIAL: the side stream's passes run on s, in the same order
  const hipStream_t side = (A->profiling & FMM_PROFILE_SERIAL) ? s : A->aux;
  const int order = A->tune.pair_order;
  // orders 3 and 4 with near_early: the shortest items (the tail of the item list)
  // on a second side stream from the start, on a small grid of waves that
  // loop over them, beside the upward passes and the M2L
  const int nit = A->dt.nitems;
  const int nearly = near_early_items(A->tune, nit, far);
  const int nmain = nit - nearly;
  const hipStream_t side2 = (A->profiling & FMM_PROFILE_SERIAL) ? s : A->aux2;
  const hipStream_t side3 = (A->profiling & FMM_PROFILE_SERIAL) ? s : A->aux3;
  auto early = [&](hipEvent_t after) -> int {
    FMM_HIP_TRY(hipStreamWaitEvent(side2, after, 0));
    int r = near(side2, nmain, nearly, std::min(nearly, A->tune.near_early_grid), FMM_PHASE_NEAR_EARLY);
    if (r) return r;
    FMM_HIP_TRY(hipEventRecord(A->ev_near, side2));
    return FMM_OK;
  };
  if (far && order == 4) {
    // order 4: the path that bounds the step stays on s with no wait across
    // streams (P2M, UT, M2M, M2L, then the main near items); P2L, its
    // projection and the M2P sources run on the side stream once P2M is
    // done, and the downward pass there once the M2L is done
    FMM_HIP_TRY(hipEventRecord(A->ev_fork, s));
    if (nearly > 0 && !A->tune.near_early_start && (rc = early(A->ev_fork))) return rc;
    if ((rc = eval_passes_pair<T, NR>(A, B, s, 1, B->ev_fork, A->ev_up, dips, true, side3))) return rc;
    if (nearly > 0 && A->tune.near_early_start && (rc = early(B->ev_fork))) return rc;
    FMM_HIP_TRY(hipEventRecord(A->ev_m2l, s));
    FMM_HIP_TRY(hipStreamWaitEvent(side, B->ev_fork, 0));
    if ((rc = pair_off_chain<T, NR>(A, B, side, dips, true, true))) return rc;
    FMM_HIP_TRY(hipStreamWaitEvent(side, A->ev_m2l, 0));
    if ((rc = eval_passes_pair<T, NR>(A, B, side, 2, nullptr, nullptr, dips))) return rc;
    if (nearly > 0) FMM_HIP_TRY(hipStreamWaitEvent(side, A->ev_near, 0));
    FMM_HIP_TRY(hipEventRecord(A->ev_join, side));
    if ((rc = near(s, 0, nmain, nmain, FMM_PHASE_NEAR))) return rc;
    FMM_HIP_TRY(hipStreamWaitEvent(s, A->ev_join, 0));
    return FMM_OK;
  }
  if (far) {
    FMM_HIP_TRY(hipEventRecord(A->ev_fork, s));
    FMM_HIP_TRY(hipStreamWaitEvent(side, A->ev_fork, 0));
    // the early items start with the passes (near_early_start 0) or once
    // P2M is done (1: P2M, VALU work at the head of the upward pass, then
    // has the GPU to itself)
    if (nearly > 0 && !A->tune.near_early_start && (rc = early(A->ev_fork))) return rc;
    if ((rc = eval_passes_pair<T, NR>(A, B, side, 1, B->ev_fork, A->ev_up, dips, true, side3))) return rc;
    if (nearly > 0 && A->tune.near_early_start && (rc = early(B->ev_fork))) return rc;
    if (order == 3) FMM_HIP_TRY(hipEventRecord(A->ev_m2l, side));
    // the near field starts once P2M (VALU, like the near field) is done and
    // shares the GPU with the GEMM passes; P2L and its projection (which the
    // M2L sums wait for) run after it (order 0) or before it (1: the near
    // field then also waits for the upward pass; 2: it does not; 3: it
    // waits for the M2L, so that the upward pass and the M2L have the GPU to
    // themselves and the near field shares it with the downward pass)
    FMM_HIP_TRY(hipStreamWaitEvent(s, B->ev_fork, 0));
    if (order == 3) {
      // P2L, its projection and the M2P sources' equivalent densities beside
      // the upward GEMMs and the M2L
      if ((rc = pair_off_chain<T, NR>(A, B, s, dips, true, true))) return rc;
      FMM_HIP_TRY(hipStreamWaitEvent(s, A->ev_m2l, 0));
    } else if (order != 0) {
      if ((rc = pair_p2l_proj<T, NR>(A, B, s, dips))) return rc;
      if (order == 1) FMM_HIP_TRY(hipStreamWaitEvent(s, A->ev_up, 0));
    }
  }
  if ((rc = near(s, 0, nmain, nmain, FMM_PHASE_NEAR))) return rc;
  if (far) {
    if (order != 3 && (rc = pair_off_chain<T, NR>(A, B, s, dips, order == 0))) return rc;
    FMM_HIP_TRY(hipStreamWaitEvent(side, B->ev_join, 0));
    if ((rc = eval_passes_pair<T, NR>(A, B, side, 2, nullptr, nullptr, dips))) return rc;
    // the side stream takes in the early launch (done long before the
    // downward pass ends), so that s waits on one event before the far field
    if (nearly > 0) FMM_HIP_TRY(hipStreamWaitEvent(side, A->ev_near, 0));
    FMM_HIP_TRY(hipEventRecord(A->ev_join, side));
    FMM_HIP_TRY(hipStreamWaitEvent(s, A->ev_join, 0));
  }
  return FMM_OK;
}

template <typename T, int NR>
static int eval_pair_chunk(fmm_plan *A, fmm_plan *B, const T *q, T *pot_a, T *grad_a, T *pot_b, T *grad_b,
                           hipStream_t s) {
  const DevTree &D = A->dt;
  const int64_t N = A->n;
  int rc;
  if ((rc = eval_permute<T, NR>(A, q, s))) return rc;
  const T kappa = (T)B->kappa;
  const T scale = (T)(1.0 / (4.0 * M_PI));
  T *acc = (T *)A->pair_acc;
  auto near = [&](hipStream_t st, int i0, int cnt, int grid, int phase) -> int {
    if (cnt <= 0) return FMM_OK;
    hipEvent_t eb, ee;
    prof_launch(A, phase, &eb, &ee);
    hipExtLaunchKernelGGL((k_near_pair<T, NR>), dim3(grid), dim3(64), A->tune.near_lds, st, eb, ee, 0, D.items,
                          D.leaves, (const T *)D.pts, (const T *)A->qs, N, D.box_begin, D.box_end, D.near_off,
                          D.near_rng, (const T *)D.near_o, acc, kappa, cnt, i0);
    FMM_HIP_TRY(hipGetLastError());
    return FMM_OK;
  };

  if (A->tune.gemm_chain && D.maxlevel >= 2 && (rc = ensure_chains<T, NR>(A, B))) return rc;
  if ((rc = pair_fork_join<T, NR>(A, B, s, (const T *)nullptr, near))) return rc;
  hipEvent_t ev = prof_begin(A, FMM_PHASE_FAR, s);
  if (D.nitems > 0)
    hipLaunchKernelGGL((k_far_pair<T, NR, true>), dim3(D.nitems), dim3(64), 0, s, D.items, D.leaves, (const T *)D.pts, N,
                       D.box_begin, D.box_end, (const T *)A->surf, A->nsurf, A->ld, D.far_off, D.far_idx,
                       (const T *)D.far_o, (const T *)acc, (const T *)A->equ, (const T *)A->eqd, (const T *)B->equ,
                       (const T *)B->eqd, (T *)D.parts, (T *)B->dt.parts, D.perm, pot_a, grad_a, pot_b, grad_b, kappa,
                       scale);
  if (D.nsplit > 0) {
    hipLaunchKernelGGL((k_leaf_parts<T, NR>), dim3(D.nsplit, 2), dim3(64), 0, s, D.split_tiles, D.leaves,
                       D.box_begin, D.box_end, (const T *)D.parts, D.perm, N, pot_a, grad_a, scale,
                       (const T *)B->dt.parts, pot_b, grad_b);
  }
  FMM_HIP_TRY(hipGetLastError());
  prof_end(A, FMM_PHASE_FAR, ev, s);
  return FMM_OK;
}

template <typename T>
static int eval_pair_typed(fmm_plan *A, fmm_plan *B, const T *q, int nrhs, T *pot_a, T *grad_a, T *pot_b, T *grad_b,
                           hipStream_t s) {
  const int64_t N = A->n;
  for (int c0 = 0; c0 < nrhs; c0 += MAX_NR) {
    const int nr = std::min(MAX_NR, nrhs - c0);
    int rc;
    if ((rc = ensure_work(A, nr)) || (rc = ensure_lists(A, nr)) || (rc = ensure_work(B, nr)) ||
        (rc = ensure_lists(B, nr)) || (rc = ensure_pair(A, B, nr)))
      return rc;
    const T *qc = q + (int64_t)c0 * N;
    T *pa = pot_a + (int64_t)c0 * N, *pb = pot_b + (int64_t)c0 * N;
    T *ga = grad_a ? grad_a + (int64_t)c0 * N * 3 : nullptr;
    T *gb = grad_b ? grad_b + (int64_t)c0 * N * 3 : nullptr;
    switch (nr) {
      case 1: rc = eval_pair_chunk<T, 1>(A, B, qc, pa, ga, pb, gb, s); break;
      case 2: rc = eval_pair_chunk<T, 2>(A, B, qc, pa, ga, pb, gb, s); break;
      case 3: rc = eval_pair_chunk<T, 3>(A, B, qc, pa, ga, pb, gb, s); break;
      default: rc = eval_pair_chunk<T, 4>(A, B, qc, pa, ga, pb, gb, s); break;
    }
    if (rc) return rc;
  }
  return FMM_OK;
}

int eval_pair_dispatch(fmm_plan *A, fmm_plan *B, const void *q, int nrhs, void *pot_a, void *grad_a, void *pot_b,
                       void *grad_b, hipStream_t s) {
  if (A->precision == FMM_FP64)
    return eval_pair_typed<double>(A, B, (const double *)q, nrhs, (double *)pot_a, (double *)grad_a, (double *)pot_b,
                                   (double *)grad_b, s);
  return eval_pair_typed<float>(A, B, (const float *)q, nrhs, (float *)pot_a, (float *)grad_a, (float *)pot_b,
                                (float *)grad_b, s);
}

int ensure_pair_md(fmm_plan *A, fmm_plan *B);  // host: the permuted dipole records

// Pair evaluation with monopole + dipole sources, potentials only (one
// column); the same stream layout as eval_pair_chunk.
template <typename T>
static int eval_pair_md_typed(fmm_plan *A, fmm_plan *B, const T *q, const T *dip, T ca, T cb, T *pot_a, T *grad_a,
                              T *pot_b, T *grad_b, hipStream_t s) {
  const bool grad = grad_a || grad_b;
  int rc;
  if ((rc = ensure_work(A, 1)) || (rc = ensure_lists(A, 1)) || (rc = ensure_work(B, 1)) ||
      (rc = ensure_lists(B, 1)) || (rc = ensure_pair(A, B, 1)) || (rc = ensure_pair_md(A, B)))
    return rc;
  const DevTree &D = A->dt;
  const int64_t N = A->n;
  T *dips = (T *)A->dips;
  hipEvent_t ev = prof_begin(A, FMM_PHASE_PERMUTE, s);
  hipLaunchKernelGGL(k_permute_md<T>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, q, dip, D.perm, N, ca, cb,
                     (T *)D.pts, dips);
  FMM_HIP_TRY(hipGetLastError());
  prof_end(A, FMM_PHASE_PERMUTE, ev, s);
  const T kappa = (T)B->kappa;
  const T scale = (T)(1.0 / (4.0 * M_PI));
  T *acc = (T *)A->pair_acc;
  auto near = [&](hipStream_t st, int i0, int cnt, int grid, int phase) -> int {
    if (cnt <= 0) return FMM_OK;
    hipEvent_t eb, ee;
    prof_launch(A, phase, &eb, &ee);
    if (grad)
      hipExtLaunchKernelGGL((k_near_pair_md<T, true>), dim3(grid), dim3(64), A->tune.near_lds, st, eb, ee, 0, D.items,
                            D.leaves, (const T *)D.pts, (const T *)dips, D.box_begin, D.box_end, D.near_off,
                            D.near_rng, (const T *)D.near_o, acc, kappa, cnt, i0);
    else
      hipExtLaunchKernelGGL((k_near_pair_md<T, false>), dim3(grid), dim3(64), A->tune.near_lds, st, eb, ee, 0,
                            D.items, D.leaves, (const T *)D.pts, (const T *)dips, D.box_begin, D.box_end, D.near_off,
                            D.near_rng, (const T *)D.near_o, acc, kappa, cnt, i0);
    FMM_HIP_TRY(hipGetLastError());
    return FMM_OK;
  };
  if (A->tune.gemm_chain && D.maxlevel >= 2 && (rc = ensure_chains<T, 1>(A, B))) return rc;
  if ((rc = pair_fork_join<T, 1>(A, B, s, (const T *)dips, near))) return rc;
  ev = prof_begin(A, FMM_PHASE_FAR, s);
  if (D.nitems > 0 && grad)
    hipLaunchKernelGGL((k_far_pair<T, 1, true>), dim3(D.nitems), dim3(64), 0, s, D.items, D.leaves, (const T *)D.pts,
                       N, D.box_begin, D.box_end, (const T *)A->surf, A->nsurf, A->ld, D.far_off, D.far_idx,
                       (const T *)D.far_o, (const T *)acc, (const T *)A->equ, (const T *)A->eqd, (const T *)B->equ,
                       (const T *)B->eqd, (T *)D.parts, (T *)B->dt.parts, D.perm, pot_a, grad_a, pot_b, grad_b,
                       kappa, scale);
  else if (D.nitems > 0)
    hipLaunchKernelGGL((k_far_pair<T, 1, false>), dim3(D.nitems), dim3(64), 0, s, D.items, D.leaves, (const T *)D.pts,
                       N, D.box_begin, D.box_end, (const T *)A->surf, A->nsurf, A->ld, D.far_off, D.far_idx,
                       (const T *)D.far_o, (const T *)acc, (const T *)A->equ, (const T *)A->eqd, (const T *)B->equ,
                       (const T *)B->eqd, (T *)D.parts, (T *)B->dt.parts, D.perm, pot_a, (T *)nullptr, pot_b,
                       (T *)nullptr, kappa, scale);
  if (D.nsplit > 0) {
    hipLaunchKernelGGL((k_leaf_parts<T, 1>), dim3(D.nsplit, 2), dim3(64), 0, s, D.split_tiles, D.leaves,
                       D.box_begin, D.box_end, (const T *)D.parts, D.perm, N, pot_a, grad_a, scale,
                       (const T *)B->dt.parts, pot_b, grad_b);
  }
  FMM_HIP_TRY(hipGetLastError());
  prof_end(A, FMM_PHASE_FAR, ev, s);
  return FMM_OK;
}

int eval_pair_md_dispatch(fmm_plan *A, fmm_plan *B, const void *q, const void *dip, double ca, double cb, void *pot_a,
                          void *grad_a, void *pot_b, void *grad_b, hipStream_t s) {
  if (A->precision == FMM_FP64)
    return eval_pair_md_typed<double>(A, B, (const double *)q, (const double *)dip, ca, cb, (double *)pot_a,
                                      (double *)grad_a, (double *)pot_b, (double *)grad_b, s);
  return eval_pair_md_typed<float>(A, B, (const float *)q, (const float *)dip, (float)ca, (float)cb, (float *)pot_a,
                                   (float *)grad_a, (float *)pot_b, (float *)grad_b, s);
}

// dxyz_k = sum_c gbar_ck gphi_ck + q_ck gpsi_ck  (c over density columns)
template <typename T>
__global__ void k_adjoint_combine(int64_t N, int nrhs, const T *__restrict__ q, const T *__restrict__ gbar,
                                  const T *__restrict__ gphi, const T *__restrict__ gpsi, T *__restrict__ dx) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= N) return;
  T a0 = 0, a1 = 0, a2 = 0;
  for (int c = 0; c < nrhs; ++c) {
    const int64_t j = (int64_t)c * N + i;
    const T gb = gbar[j], qq = q[j];
    a0 += gb * gphi[3 * j] + qq * gpsi[3 * j];
    a1 += gb * gphi[3 * j + 1] + qq * gpsi[3 * j + 1];
    a2 += gb * gphi[3 * j + 2] + qq * gpsi[3 * j + 2];
  }
  dx[3 * i] = a0;
  dx[3 * i + 1] = a1;
  dx[3 * i + 2] = a2;
}

int adjoint_combine(fmm_plan *P, int nrhs, const void *q, const void *gbar, const void *gphi, const void *gpsi,
                    void *dx, hipStream_t s) {
  const int64_t N = P->n;
  if (P->precision == FMM_FP64)
    hipLaunchKernelGGL(k_adjoint_combine<double>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, nrhs,
                       (const double *)q, (const double *)gbar, (const double *)gphi, (const double *)gpsi,
                       (double *)dx);
  else
    hipLaunchKernelGGL(k_adjoint_combine<float>, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, nrhs,
                       (const float *)q, (const float *)gbar, (const float *)gphi, (const float *)gpsi, (float *)dx);
  FMM_HIP_TRY(hipGetLastError());
  return FMM_OK;
}

int eval_dispatch(fmm_plan *P, const void *q, int nrhs, void *pot, void *grad, hipStream_t s) {
  if (P->precision == FMM_FP64) return eval_typed<double>(P, (const double *)q, nrhs, (double *)pot, (double *)grad, s);
  return eval_typed<float>(P, (const float *)q, nrhs, (float *)pot, (float *)grad, s);
}

}  // namespace fmm

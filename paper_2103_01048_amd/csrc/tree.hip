// Octree levels and U/V/W/X interaction lists built on the device from the
// sorted Morton keys (Methods, fast multipole method: the enclosing cube is
// split until a leaf holds at most a constant number of points; the near
// field and the interaction list of each box).
//
// Levels: a box at level l splits while it holds more than ncrit points and
// l < 21.  Its children are the runs of equal level-(l+1) key prefixes among
// its points, so one pass over the points flags every run start, an
// inclusive scan numbers the new boxes in point order, which is the order
// (level, molecule, key) of the boxes, and each point moves to its child.
//
// Lists of an adaptive tree (B a box at level l, "adjacent" = closed cubes
// touching):
//   V(B), l >= 2: children of the 27 same-level boxes around B's parent
//                 that are not adjacent to B;
//   U(B), leaf:   for each of the 27 cells around B, the deepest existing
//                 box containing the cell if it is a leaf (B itself
//                 included), or, for a same-level box with children, its
//                 leaf descendants adjacent to B;
//   W(B), leaf:   descendants of same-level neighbours that are not adjacent
//                 to B but whose parent is;
//   X(B):         the boxes A with B in W(A).
// Each list is produced in two passes (count, then fill at scanned offsets)
// and sorted per box with a segmented radix sort, which gives the ascending
// order the host planner used.  Every integer result equals the host build.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include "fmm_internal.h"

namespace fmm {

namespace {

struct LevelIndex {
  int32_t begin[MAXLEVEL + 2];  // boxes of level l: [begin[l], begin[l + 1])
  int32_t nlevel;
};

constexpr int DFS_STACK = 160;  // 1 + 7 per level below a box is enough for 21 levels

__device__ inline uint64_t level_prefix(uint64_t key, int l) { return key >> (3 * (MAXLEVEL - l)); }

__device__ inline uint64_t interleave_level(int64_t x, int64_t y, int64_t z, int l) {
  uint64_t k = 0;
  for (int b = 0; b < l; ++b) {
    k |= (uint64_t)((x >> b) & 1) << (3 * b + 2);
    k |= (uint64_t)((y >> b) & 1) << (3 * b + 1);
    k |= (uint64_t)((z >> b) & 1) << (3 * b);
  }
  return k;
}

__global__ void k_tree_fill(int32_t *__restrict__ a, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) a[i] = v;
}

// pbox[i] = root box of the molecule holding point i (mol_off: nmol + 1
// point offsets, root: per molecule its root box or -1 when empty)
__global__ void k_tree_roots(int64_t n, const int64_t *__restrict__ mol_off, int nmol,
                             const int32_t *__restrict__ root, int32_t *__restrict__ pbox) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= n) return;
  int lo = 0, hi = nmol;  // last molecule m with mol_off[m] <= i
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (mol_off[mid] <= i) lo = mid;
    else hi = mid;
  }
  pbox[i] = root[lo];
}

// Run starts of the children of every box at level l that splits; points
// of boxes that do not split leave the build (pbox = -1).
__global__ void k_tree_flags(const uint64_t *__restrict__ keys, int64_t n, int l, int ncrit,
                             int32_t *__restrict__ pbox, const int32_t *__restrict__ bbeg,
                             const int32_t *__restrict__ bend, int32_t *__restrict__ flag) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= n) return;
  const int b = pbox[i];
  int f = 0;
  if (b >= 0) {
    if (bend[b] - bbeg[b] > ncrit && l < MAXLEVEL) {
      f = (i == bbeg[b]) || (level_prefix(keys[i], l + 1) != level_prefix(keys[i - 1], l + 1));
    } else {
      pbox[i] = -1;
    }
  }
  flag[i] = f;
}

// New boxes numbered base + (inclusive count of run starts) - 1; every point
// of a splitting box moves to its child.
__global__ void k_tree_children(const uint64_t *__restrict__ keys, int64_t n, int l, int32_t base,
                                const int32_t *__restrict__ flag, const int32_t *__restrict__ scan,
                                int32_t *__restrict__ pbox, int32_t *__restrict__ bbeg, int32_t *__restrict__ bpar,
                                uint64_t *__restrict__ bpre, int32_t *__restrict__ bmol, int32_t *__restrict__ blev) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= n) return;
  const int b = pbox[i];
  if (b < 0) return;
  const int c = base + scan[i] - 1;
  if (flag[i]) {
    bbeg[c] = (int32_t)i;
    bpar[c] = b;
    bpre[c] = level_prefix(keys[i], l + 1);
    bmol[c] = bmol[b];
    blev[c] = l + 1;
  }
  pbox[i] = c;
}

// End of each new box (the next sibling's begin or the parent's end) and
// the parent's first child and child count.
__global__ void k_tree_links(int32_t c0, int32_t c1, const int32_t *__restrict__ bbeg, int32_t *__restrict__ bend,
                             const int32_t *__restrict__ bpar, int32_t *__restrict__ cbeg,
                             int32_t *__restrict__ nch) {
  const int32_t c = c0 + (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (c >= c1) return;
  const int p = bpar[c];
  bend[c] = (c + 1 < c1 && bpar[c + 1] == p) ? bbeg[c + 1] : bend[p];
  if (c == c0 || bpar[c - 1] != p) cbeg[p] = c;
  atomicAdd(&nch[p], 1);
}

__global__ void k_tree_anchor(int32_t nb, const uint64_t *__restrict__ bpre, const int32_t *__restrict__ blev,
                              int32_t *__restrict__ anc) {
  const int32_t b = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (b >= nb) return;
  const int l = blev[b];
  const uint64_t pre = bpre[b];
  int32_t a[3] = {0, 0, 0};
  for (int k = 0; k < l; ++k) {
    const uint64_t dig = (pre >> (3 * (l - 1 - k))) & 7;
    a[0] = (a[0] << 1) | (int32_t)((dig >> 2) & 1);
    a[1] = (a[1] << 1) | (int32_t)((dig >> 1) & 1);
    a[2] = (a[2] << 1) | (int32_t)(dig & 1);
  }
  anc[3 * b] = a[0];
  anc[3 * b + 1] = a[1];
  anc[3 * b + 2] = a[2];
}

struct TreeView {
  LevelIndex L;
  const uint64_t *pre;
  const int32_t *mol, *lev, *anc, *par, *cbeg, *nch;
};

// Box of molecule `mol` at level l with integer coordinates (x, y, z), or -1.
__device__ int32_t tree_find(const TreeView &t, int mol, int l, int64_t x, int64_t y, int64_t z) {
  if (l >= t.L.nlevel) return -1;
  const int64_t side = (int64_t)1 << l;
  if (x < 0 || y < 0 || z < 0 || x >= side || y >= side || z >= side) return -1;
  const uint64_t key = interleave_level(x, y, z, l);
  int32_t lo = t.L.begin[l], hi = t.L.begin[l + 1];
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (t.mol[mid] < mol || (t.mol[mid] == mol && t.pre[mid] < key)) lo = mid + 1;
    else hi = mid;
  }
  return (lo < t.L.begin[l + 1] && t.mol[lo] == mol && t.pre[lo] == key) ? lo : -1;
}

__device__ bool tree_adjacent(const TreeView &t, int32_t a, int32_t b) {
  const int64_t sa = (int64_t)1 << (MAXLEVEL - t.lev[a]), sb = (int64_t)1 << (MAXLEVEL - t.lev[b]);
  for (int d = 0; d < 3; ++d) {
    const int64_t loa = (int64_t)t.anc[3 * a + d] * sa, lob = (int64_t)t.anc[3 * b + d] * sb;
    if (loa > lob + sb || lob > loa + sa) return false;
  }
  return true;
}

// V lists: count (off == nullptr) or fill.
__global__ void k_list_v(int32_t nb, TreeView t, int32_t *__restrict__ cnt, const int64_t *__restrict__ off,
                         int32_t *__restrict__ out) {
  const int32_t b = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (b >= nb) return;
  const int l = t.lev[b];
  int32_t k = 0;
  if (l >= 2) {
    const int32_t p = t.par[b];
    const int64_t px = t.anc[3 * p], py = t.anc[3 * p + 1], pz = t.anc[3 * p + 2];
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          const int32_t c = tree_find(t, t.mol[b], l - 1, px + dx, py + dy, pz + dz);
          if (c < 0) continue;
          for (int j = 0; j < t.nch[c]; ++j) {
            const int32_t ch = t.cbeg[c] + j;
            if (tree_adjacent(t, ch, b)) continue;
            if (off) out[off[b] + k] = ch;
            ++k;
          }
        }
  }
  if (!off) cnt[b] = k;
}

// U and W lists of the leaves: count (offU == nullptr) or fill.  A stack
// overflow (a box with more levels of adjacent descendants than the stack
// holds) sets *overflow; the host then builds the lists itself.
__global__ void k_list_uw(int32_t nb, TreeView t, int32_t *__restrict__ cntU, int32_t *__restrict__ cntW,
                          const int64_t *__restrict__ offU, const int64_t *__restrict__ offW,
                          int32_t *__restrict__ outU, int32_t *__restrict__ outW, int32_t *__restrict__ overflow) {
  const int32_t b = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (b >= nb) return;
  int32_t ku = 0, kw = 0;
  if (t.nch[b] == 0) {
    const int l = t.lev[b], mol = t.mol[b];
    const int64_t ax = t.anc[3 * b], ay = t.anc[3 * b + 1], az = t.anc[3 * b + 2];
    int32_t coarse[27];  // leaves found at a coarser level (found from several cells)
    int ncoarse = 0;
    int32_t stk[DFS_STACK];
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          int64_t cx = ax + dx, cy = ay + dy, cz = az + dz;
          const int64_t side = (int64_t)1 << l;
          if (cx < 0 || cy < 0 || cz < 0 || cx >= side || cy >= side || cz >= side) continue;
          int ll = l;
          int32_t box = -1;
          while (ll >= 0) {
            box = tree_find(t, mol, ll, cx, cy, cz);
            if (box >= 0) break;
            --ll;
            cx >>= 1;
            cy >>= 1;
            cz >>= 1;
          }
          if (box < 0) continue;
          if (t.nch[box] == 0) {
            if (ll < l) {
              bool seen = false;
              for (int q = 0; q < ncoarse; ++q) seen |= coarse[q] == box;
              if (seen) continue;
              coarse[ncoarse++] = box;
            }
            if (offU) outU[offU[b] + ku] = box;
            ++ku;
          } else if (ll == l) {
            int sp = 0;
            for (int j = t.nch[box] - 1; j >= 0; --j) stk[sp++] = t.cbeg[box] + j;
            while (sp > 0) {
              const int32_t d = stk[--sp];
              if (tree_adjacent(t, d, b)) {
                if (t.nch[d] == 0) {
                  if (offU) outU[offU[b] + ku] = d;
                  ++ku;
                } else {
                  if (sp + t.nch[d] > DFS_STACK) {
                    atomicExch(overflow, 1);
                    sp = 0;
                    break;
                  }
                  for (int j = t.nch[d] - 1; j >= 0; --j) stk[sp++] = t.cbeg[d] + j;
                }
              } else {
                if (offW) outW[offW[b] + kw] = d;
                ++kw;
              }
            }
          }
        }
  }
  if (!offU) {
    cntU[b] = ku;
    cntW[b] = kw;
  }
}

// X lists, the transpose of W: counts, then entries at atomic cursors (the
// order is fixed afterwards by the segmented sort).
__global__ void k_list_xcount(int32_t nb, const int64_t *__restrict__ offW, const int32_t *__restrict__ W,
                              int32_t *__restrict__ cntX) {
  const int32_t b = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (b >= nb) return;
  for (int64_t k = offW[b]; k < offW[b + 1]; ++k) atomicAdd(&cntX[W[k]], 1);
}

__global__ void k_list_xfill(int32_t nb, const int64_t *__restrict__ offW, const int32_t *__restrict__ W,
                             const int64_t *__restrict__ offX, int32_t *__restrict__ cur, int32_t *__restrict__ X) {
  const int32_t b = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (b >= nb) return;
  for (int64_t k = offW[b]; k < offW[b + 1]; ++k) {
    const int32_t a = W[k];
    X[offX[a] + atomicAdd(&cur[a], 1)] = b;
  }
}

// off[0] = 0, off[b + 1] = off[b] + cnt[b]
__global__ void k_counts_to_i64(int32_t n, const int32_t *__restrict__ cnt, int64_t *__restrict__ c64) {
  const int32_t b = (int32_t)(blockIdx.x * 256 + threadIdx.x);
  if (b < n) c64[b] = cnt[b];
}

inline unsigned blocks_of(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

// Device allocations of the build, released at the end of device_tree.
struct Scratch {
  std::vector<void *> ptrs;
  ~Scratch() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  hipError_t get(T **p, size_t count) {
    void *q = nullptr;
    const hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
    if (e == hipSuccess) ptrs.push_back(q);
    *p = (T *)q;
    return e;
  }
};

#define TREE_TRY(call)                                                                   \
  do {                                                                                   \
    const hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                              \
      set_error(std::string("device tree: ") + #call + ": " + hipGetErrorString(e_));    \
      return FMM_EHIP;                                                                   \
    }                                                                                    \
  } while (0)

// offsets (nb + 1, int64) from counts; the CSR total on the host
int scan_offsets(Scratch &S, int32_t nb, const int32_t *cnt, int64_t **off, int64_t *total, hipStream_t s) {
  int64_t *c64 = nullptr;
  TREE_TRY(S.get(&c64, (size_t)nb + 1));
  TREE_TRY(S.get(off, (size_t)nb + 1));
  hipLaunchKernelGGL(k_counts_to_i64, dim3(blocks_of(nb)), dim3(256), 0, s, nb, cnt, c64);
  TREE_TRY(hipMemsetAsync(*off, 0, sizeof(int64_t), s));
  size_t tmp_bytes = 0;
  TREE_TRY(rocprim::inclusive_scan(nullptr, tmp_bytes, c64, *off + 1, (size_t)nb, rocprim::plus<int64_t>(), s));
  void *tmp = nullptr;
  TREE_TRY(S.get((char **)&tmp, tmp_bytes));
  TREE_TRY(rocprim::inclusive_scan(tmp, tmp_bytes, c64, *off + 1, (size_t)nb, rocprim::plus<int64_t>(), s));
  TREE_TRY(hipMemcpyAsync(total, *off + nb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  TREE_TRY(hipStreamSynchronize(s));
  return FMM_OK;
}

// Sort each box's entries ascending (keys in place through a second buffer).
int sort_segments(Scratch &S, int32_t nb, const int64_t *off, int32_t *vals, int64_t total, hipStream_t s) {
  if (total <= 1) return FMM_OK;
  int32_t *tmpk = nullptr;
  TREE_TRY(S.get(&tmpk, (size_t)total));
  size_t tmp_bytes = 0;
  TREE_TRY(rocprim::segmented_radix_sort_keys(nullptr, tmp_bytes, vals, tmpk, (unsigned)total, (unsigned)nb, off,
                                              off + 1, 0, 32, s));
  void *tmp = nullptr;
  TREE_TRY(S.get((char **)&tmp, tmp_bytes));
  TREE_TRY(rocprim::segmented_radix_sort_keys(tmp, tmp_bytes, vals, tmpk, (unsigned)total, (unsigned)nb, off, off + 1,
                                              0, 32, s));
  TREE_TRY(hipMemcpyAsync(vals, tmpk, (size_t)total * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  return FMM_OK;
}

template <typename A, typename B>
void widen(const std::vector<A> &in, std::vector<B> &out) {
  out.resize(in.size());
  for (size_t i = 0; i < in.size(); ++i) out[i] = (B)in[i];
}

}  // namespace

// Octree and lists of plan P on the device from the sorted keys d_keys
// (device, P->n values, molecules in P->mol_off order).  Fills the host
// arrays of P (boxes by (level, molecule, key); U, V, W, X in CSR).  Returns
// FMM_OK, or 1 when the U/W traversal overflowed its stack (P's tree
// arrays are then filled and its lists are not).
int device_tree(fmm_plan *P, const uint64_t *d_keys, hipStream_t s, double *ms_tree, double *ms_lists) {
  const int64_t n = P->n;
  const int nmol = (int)P->mol_off.size() - 1;
  const int ncrit = P->ncrit;
  Scratch S;
  auto t0 = std::chrono::steady_clock::now();
  // roots: one per non-empty molecule
  std::vector<int32_t> h_root(nmol, -1), r_beg, r_end, r_mol;
  for (int m = 0; m < nmol; ++m)
    if (P->mol_off[m + 1] > P->mol_off[m]) {
      h_root[m] = (int32_t)r_beg.size();
      r_beg.push_back((int32_t)P->mol_off[m]);
      r_end.push_back((int32_t)P->mol_off[m + 1]);
      r_mol.push_back(m);
    }
  int64_t cap = std::max<int64_t>(1024, 4 * n / std::max(1, ncrit) + 2 * (int64_t)r_beg.size() + 64);
  int32_t *bbeg = nullptr, *bend = nullptr, *bpar = nullptr, *bmol = nullptr, *blev = nullptr, *cbeg = nullptr,
          *nch = nullptr;
  uint64_t *bpre = nullptr;
  // box arrays (grown by copying when a level needs more room)
  auto grow = [&](int64_t used, int64_t need) -> int {
    if (need <= cap && bbeg) return FMM_OK;
    const int64_t nc = std::max(need, 2 * cap);
    int32_t *a[7];
    uint64_t *pp = nullptr;
    for (int k = 0; k < 7; ++k) TREE_TRY(S.get(&a[k], (size_t)nc));
    TREE_TRY(S.get(&pp, (size_t)nc));
    hipLaunchKernelGGL(k_tree_fill, dim3(blocks_of(nc)), dim3(256), 0, s, a[5], nc, -1);
    hipLaunchKernelGGL(k_tree_fill, dim3(blocks_of(nc)), dim3(256), 0, s, a[6], nc, 0);
    if (bbeg && used > 0) {
      int32_t *old[7] = {bbeg, bend, bpar, bmol, blev, cbeg, nch};
      for (int k = 0; k < 7; ++k)
        TREE_TRY(hipMemcpyAsync(a[k], old[k], (size_t)used * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
      TREE_TRY(hipMemcpyAsync(pp, bpre, (size_t)used * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
    }
    bbeg = a[0]; bend = a[1]; bpar = a[2]; bmol = a[3]; blev = a[4]; cbeg = a[5]; nch = a[6]; bpre = pp;
    cap = nc;
    return FMM_OK;
  };
  int rc;
  if ((rc = grow(0, cap))) return rc;
  const int32_t nroot = (int32_t)r_beg.size();
  {
    std::vector<int32_t> zero(nroot, 0), minus(nroot, -1);
    std::vector<uint64_t> zp(nroot, 0);
    TREE_TRY(hipMemcpyAsync(bbeg, r_beg.data(), nroot * sizeof(int32_t), hipMemcpyHostToDevice, s));
    TREE_TRY(hipMemcpyAsync(bend, r_end.data(), nroot * sizeof(int32_t), hipMemcpyHostToDevice, s));
    TREE_TRY(hipMemcpyAsync(bpar, minus.data(), nroot * sizeof(int32_t), hipMemcpyHostToDevice, s));
    TREE_TRY(hipMemcpyAsync(bmol, r_mol.data(), nroot * sizeof(int32_t), hipMemcpyHostToDevice, s));
    TREE_TRY(hipMemcpyAsync(blev, zero.data(), nroot * sizeof(int32_t), hipMemcpyHostToDevice, s));
    TREE_TRY(hipMemcpyAsync(bpre, zp.data(), nroot * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    TREE_TRY(hipStreamSynchronize(s));
  }
  int32_t *pbox = nullptr, *flag = nullptr, *scan = nullptr, *d_root = nullptr;
  int64_t *d_moff = nullptr;
  TREE_TRY(S.get(&pbox, (size_t)n));
  TREE_TRY(S.get(&flag, (size_t)n));
  TREE_TRY(S.get(&scan, (size_t)n));
  TREE_TRY(S.get(&d_root, (size_t)nmol));
  TREE_TRY(S.get(&d_moff, (size_t)nmol + 1));
  TREE_TRY(hipMemcpyAsync(d_root, h_root.data(), nmol * sizeof(int32_t), hipMemcpyHostToDevice, s));
  TREE_TRY(hipMemcpyAsync(d_moff, P->mol_off.data(), (nmol + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_tree_roots, dim3(blocks_of(n)), dim3(256), 0, s, n, d_moff, nmol, d_root, pbox);
  size_t scan_bytes = 0;
  TREE_TRY(rocprim::inclusive_scan(nullptr, scan_bytes, flag, scan, (size_t)n, rocprim::plus<int32_t>(), s));
  void *scan_tmp = nullptr;
  TREE_TRY(S.get((char **)&scan_tmp, scan_bytes));
  std::vector<int64_t> lb = {0, nroot};
  int32_t lvl_start = 0, lvl_end = nroot;
  for (int l = 0; l < MAXLEVEL; ++l) {
    hipLaunchKernelGGL(k_tree_flags, dim3(blocks_of(n)), dim3(256), 0, s, d_keys, n, l, ncrit, pbox, bbeg, bend,
                       flag);
    TREE_TRY(rocprim::inclusive_scan(scan_tmp, scan_bytes, flag, scan, (size_t)n, rocprim::plus<int32_t>(), s));
    int32_t total = 0;
    TREE_TRY(hipMemcpyAsync(&total, scan + (n - 1), sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TREE_TRY(hipStreamSynchronize(s));
    if (total == 0) break;
    if ((rc = grow(lvl_end, (int64_t)lvl_end + total))) return rc;
    hipLaunchKernelGGL(k_tree_children, dim3(blocks_of(n)), dim3(256), 0, s, d_keys, n, l, lvl_end, flag, scan, pbox,
                       bbeg, bpar, bpre, bmol, blev);
    hipLaunchKernelGGL(k_tree_links, dim3(blocks_of(total)), dim3(256), 0, s, lvl_end, lvl_end + total, bbeg, bend,
                       bpar, cbeg, nch);
    TREE_TRY(hipGetLastError());
    lvl_start = lvl_end;
    lvl_end += total;
    lb.push_back(lvl_end);
  }
  (void)lvl_start;
  const int32_t nb = lvl_end;
  int32_t *anc = nullptr;
  TREE_TRY(S.get(&anc, (size_t)nb * 3));
  hipLaunchKernelGGL(k_tree_anchor, dim3(blocks_of(nb)), dim3(256), 0, s, nb, bpre, blev, anc);
  TREE_TRY(hipGetLastError());
  // boxes to the host
  {
    std::vector<int32_t> h_beg(nb), h_end(nb), h_par(nb), h_mol(nb), h_lev(nb), h_cb(nb), h_nc(nb), h_anc(3 * (size_t)nb);
    TREE_TRY(hipMemcpyAsync(h_beg.data(), bbeg, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TREE_TRY(hipMemcpyAsync(h_end.data(), bend, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TREE_TRY(hipMemcpyAsync(h_par.data(), bpar, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TREE_TRY(hipMemcpyAsync(h_mol.data(), bmol, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TREE_TRY(hipMemcpyAsync(h_lev.data(), blev, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TREE_TRY(hipMemcpyAsync(h_cb.data(), cbeg, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TREE_TRY(hipMemcpyAsync(h_nc.data(), nch, nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TREE_TRY(hipMemcpyAsync(h_anc.data(), anc, 3 * (size_t)nb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TREE_TRY(hipStreamSynchronize(s));
    widen(h_beg, P->begin);
    widen(h_end, P->end);
    widen(h_par, P->parent);
    widen(h_cb, P->child_begin);
    widen(h_anc, P->anchor);
    P->nchild = h_nc;
    P->level = h_lev;
    P->mol = h_mol;
    P->level_begin = lb;
  }
  auto t1 = std::chrono::steady_clock::now();
  if (ms_tree) *ms_tree = std::chrono::duration<double, std::milli>(t1 - t0).count();
  // lists
  TreeView t;
  std::memset(&t.L, 0, sizeof(t.L));
  t.L.nlevel = (int32_t)lb.size() - 1;
  for (size_t k = 0; k < lb.size() && k < (size_t)MAXLEVEL + 2; ++k) t.L.begin[k] = (int32_t)lb[k];
  t.pre = bpre; t.mol = bmol; t.lev = blev; t.anc = anc; t.par = bpar; t.cbeg = cbeg; t.nch = nch;
  int32_t *cU = nullptr, *cV = nullptr, *cW = nullptr, *cX = nullptr, *ovf = nullptr;
  TREE_TRY(S.get(&cU, nb)); TREE_TRY(S.get(&cV, nb)); TREE_TRY(S.get(&cW, nb)); TREE_TRY(S.get(&cX, nb));
  TREE_TRY(S.get(&ovf, 1));
  hipLaunchKernelGGL(k_tree_fill, dim3(1), dim3(256), 0, s, ovf, 1, 0);
  hipLaunchKernelGGL(k_tree_fill, dim3(blocks_of(nb)), dim3(256), 0, s, cX, (int64_t)nb, 0);
  hipLaunchKernelGGL(k_list_v, dim3(blocks_of(nb)), dim3(256), 0, s, nb, t, cV, (const int64_t *)nullptr,
                     (int32_t *)nullptr);
  hipLaunchKernelGGL(k_list_uw, dim3(blocks_of(nb)), dim3(256), 0, s, nb, t, cU, cW, (const int64_t *)nullptr,
                     (const int64_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr, ovf);
  TREE_TRY(hipGetLastError());
  int32_t h_ovf = 0;
  TREE_TRY(hipMemcpyAsync(&h_ovf, ovf, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  TREE_TRY(hipStreamSynchronize(s));
  if (h_ovf) return 1;
  int64_t *oU, *oV, *oW, *oX, nU, nV, nW, nX;
  if ((rc = scan_offsets(S, nb, cU, &oU, &nU, s)) || (rc = scan_offsets(S, nb, cV, &oV, &nV, s)) ||
      (rc = scan_offsets(S, nb, cW, &oW, &nW, s)))
    return rc;
  int32_t *U, *V, *Wl, *X, *cur;
  TREE_TRY(S.get(&U, (size_t)nU)); TREE_TRY(S.get(&V, (size_t)nV)); TREE_TRY(S.get(&Wl, (size_t)nW));
  hipLaunchKernelGGL(k_list_v, dim3(blocks_of(nb)), dim3(256), 0, s, nb, t, cV, oV, V);
  hipLaunchKernelGGL(k_list_uw, dim3(blocks_of(nb)), dim3(256), 0, s, nb, t, cU, cW, oU, oW, U, Wl, ovf);
  hipLaunchKernelGGL(k_list_xcount, dim3(blocks_of(nb)), dim3(256), 0, s, nb, oW, Wl, cX);
  TREE_TRY(hipGetLastError());
  if ((rc = scan_offsets(S, nb, cX, &oX, &nX, s))) return rc;
  TREE_TRY(S.get(&X, (size_t)nX));
  TREE_TRY(S.get(&cur, nb));
  hipLaunchKernelGGL(k_tree_fill, dim3(blocks_of(nb)), dim3(256), 0, s, cur, (int64_t)nb, 0);
  hipLaunchKernelGGL(k_list_xfill, dim3(blocks_of(nb)), dim3(256), 0, s, nb, oW, Wl, oX, cur, X);
  TREE_TRY(hipGetLastError());
  if ((rc = sort_segments(S, nb, oU, U, nU, s)) || (rc = sort_segments(S, nb, oV, V, nV, s)) ||
      (rc = sort_segments(S, nb, oW, Wl, nW, s)) || (rc = sort_segments(S, nb, oX, X, nX, s)))
    return rc;
  const int64_t *offs[4] = {oU, oV, oW, oX};
  const int32_t *vals[4] = {U, V, Wl, X};
  const int64_t tot[4] = {nU, nV, nW, nX};
  std::vector<int32_t> hv;
  for (int k = 0; k < 4; ++k) {
    P->loff[k].resize((size_t)nb + 1);
    TREE_TRY(hipMemcpyAsync(P->loff[k].data(), offs[k], ((size_t)nb + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    hv.resize((size_t)tot[k]);
    TREE_TRY(hipMemcpyAsync(hv.data(), vals[k], (size_t)tot[k] * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TREE_TRY(hipStreamSynchronize(s));
    widen(hv, P->lidx[k]);
  }
  if (ms_lists) *ms_lists = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t1).count();
  return FMM_OK;
}

}  // namespace fmm

// Internal structures of the MI355X FMM library (host planner + kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/fmmbem.h"

namespace fmm {

constexpr int MAXLEVEL = 21;
constexpr int GEMM_NT = 64;   // columns per GEMM task (4 MFMA column blocks)
constexpr int MAX_NR = 4;     // density columns handled by one kernel pass

// Surface radii, in units of the box half-width (upward equivalent, upward
// check, downward equivalent, downward check).
constexpr double ALPHA_UE = 1.05, ALPHA_UC = 2.95, ALPHA_DE = 2.95, ALPHA_DC = 1.05;

void set_error(const std::string &msg);
int plan_upload(fmm_plan *P, void **ptr, const void *h, size_t bytes);
hipEvent_t prof_begin(fmm_plan *P, int phase, hipStream_t s);
void prof_end(fmm_plan *P, int phase, hipEvent_t begin, hipStream_t s);
// Timing events for a phase that is a single kernel launch: the launch
// carries them (hipExtLaunchKernelGGL), so no marker goes on the stream
// beside it.  Both null when the phase is not being timed.
void prof_launch(fmm_plan *P, int phase, hipEvent_t *begin, hipEvent_t *end);
// Near-field items of a pair evaluation that start at once on the second
// side stream: near_early per mille of the items (the shortest, at the tail
// of the item list), with pass order 3 or 4 and a far field only.
inline int near_early_items(const fmm_tuning_t &t, int nitems, bool far) {
  return (far && t.pair_order >= 3 && t.near_early > 0)
             ? (int)std::min<int64_t>(nitems, (int64_t)nitems * t.near_early / 1000)
             : 0;
}
void pinv_tsvd(int n, const double *A, double tau, double *out);
int tsvd_factors(int n, const double *A, double tau, double *UT, double *VS, int nthreads);
int tsvd_split(int rows, int cols, const double *A, double tau, double *L, int ldl, double *R, int ldr);

#define FMM_HIP_TRY(call)                                                        \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) {                                                      \
      ::fmm::set_error(std::string(#call) + ": " + hipGetErrorString(e_));       \
      return FMM_EHIP;                                                           \
    }                                                                            \
  } while (0)

// One GEMM work item: Y[dst[c]] (op)= alpha * A[mat] * concat_s X[src[c*S+s]]
// for columns c in [col0, col0 + ncol), ncol <= GEMM_NT.
struct GemmTask {
  int32_t mat;
  int32_t col0;
  int32_t ncol;
  int32_t nrb;     // 16-row blocks this task computes (0: the batch's nrb)
  int32_t klen;    // k-values this task reads (0: the batch's klen)
  double alpha;
};

enum GemmMode { GEMM_STORE = 0, GEMM_ADD = 1 };

// Everything one gather-GEMM batch needs on the device; a launch takes two
// (the second with ntask = 0 when unused) so that the same pass of two plans
// sharing a tree runs as one launch.
struct GemmArgs {
  const GemmTask *tasks;
  const void *pool;     // matrix pool (elements of the work type; uint4 units for bf16x3)
  int64_t mstride;      // one matrix, in pool units
  const int32_t *src;   // ncols*S row indices into X
  const int32_t *dst;   // ncols row indices into Y
  const void *X;
  void *Y;
  int ntask, nrb, klen, ldx, ldy, S, seg, KQ, mode, nt;
};

// A batch of GEMM tasks that can run in one launch (no two tasks write the
// same output rows).
struct GemmBatch {
  int S = 1;                   // K segments per column
  int nrb = 0;                 // 16-row blocks of A that are computed
  int klen = 0;                // K extent actually read (multiple of 16)
  int seg = 0;                 // K length of one segment (0: the work-array row length)
  int kq_stride = 0;           // 16-wide k groups per stored row block (0: row length / 16)
  int ldy = 0;                 // leading dimension of the output rows (0: the work-array row length)
  int mode = GEMM_STORE;
  int pool = 0;                // 0: matrix pool, 2: bf16x3 split pool
  int ldx = 0;                 // row length of X (0: the work-array row length)
  int nt = GEMM_NT;            // columns per task (the bf16x3 kernel also takes 2 GEMM_NT)
  int ntask = 0;
  GemmTask *d_tasks = nullptr;
  int32_t *d_src = nullptr;    // ncols*S  (row index into X, already * nr + r)
  int32_t *d_dst = nullptr;    // ncols    (row index into Y)
  int ncols = 0;
  // host copies kept until upload
  std::vector<GemmTask> h_tasks;
  std::vector<int32_t> h_src, h_dst;
};

// Per-nrhs-chunk task lists.  Row indices in the work arrays are
// box * nr + r, so the lists depend on nr.
// One task of a chained launch (k_chain): kind 0 runs GEMM task idx >> 4,
// row group idx & 15, of GemmArgs arg; kind 1 sums the M2M slots of the
// four boxes idx .. idx + 3 of ReduceArgs arg.  Tasks of phase p > 0 start
// once every task of phase p - 1 has finished.
struct ChainTask {
  int32_t kind, phase, arg, idx;
};

// Device task list of a chained launch and what it was built from.
struct Chain {
  std::vector<const void *> key;  // plans, column count and work arrays it was built for
  int ntask = 0, nphase = 0, kch = 0;
  void *tasks = nullptr, *gargs = nullptr, *rargs = nullptr, *need = nullptr;
};

struct PassLists {
  int nr = 0;
  // per level l (index l, levels >= 2), in singular coordinates c = U^T chk
  std::vector<GemmBatch> m2m;   // per-child M2M slots of the parents at level l
  GemmBatch ut_u_all;           // leaf upward check -> c_u, all levels
  std::vector<GemmBatch> l2l;   // child c_d += L2L * parent c_d (levels >= 3)
  GemmBatch vs_u;               // c_u -> upward equivalent (M2P sources), all levels
  GemmBatch ut_dx;              // P2L check -> its own c_d array (added by the M2L sums), all levels
  GemmBatch vs_d;               // c_d -> downward equivalent (leaves), all levels
  GemmBatch m2l;                // all levels, c_u -> pair slots of c_d (factored: intermediate -> slots)
  GemmBatch m2l_r;              // factored M2L: c_u -> per-pair intermediate (R factors)
  std::vector<int> m2l_t0;      // per level (0 .. maxlevel + 1): the first M2L task of that level (tasks
                                // ascend by level; entry maxlevel + 1 = the task count)
};

struct DevTree {
  int64_t n = 0;
  int nbox = 0, nleaf = 0, maxlevel = 0;
  // sorted points relative to their leaf's centre; xyz + density slot, in T
  void *pts = nullptr;
  int32_t *perm = nullptr;      // sorted -> caller index
  // boxes
  void *box_geom = nullptr;     // T4: centre xyz (relative to the molecule's root centre), half width
  int32_t *box_begin = nullptr, *box_end = nullptr;
  int32_t *leaves = nullptr;    // leaf box ids
  // leaf work items: (leaf slot, first target | split << 24, part or -1, 0)
  int32_t *items = nullptr;
  int nitems = 0;
  int32_t *near_off = nullptr;  // per item, into near_rng
  int32_t *near_rng = nullptr;  // (begin, end) point ranges of near sources, one leaf each
  void *near_o = nullptr;       // T4 per range: source leaf centre - target leaf centre
  void *far_o = nullptr;        // T4 per far entry: surface box centre - target leaf centre, radius
  int32_t *far_off = nullptr;   // per item, into far_idx
  int32_t *far_idx = nullptr;   // surface boxes (bit 30: own downward surface)
  int32_t *split_tiles = nullptr;  // (slot, code, first part, nparts) per split tile
  int nsplit = 0, nparts = 0;
  void *parts = nullptr;        // partial sums of split tiles
  int32_t *x_box = nullptr;     // boxes with a non-empty X list
  int32_t *x_off = nullptr, *x_idx = nullptr;
  void *x_o = nullptr;          // T4 per X entry: source leaf centre - target box centre
  int nxbox = 0;
  int32_t *v_tgt = nullptr;     // boxes at level >= 2 (M2L sums)
  int32_t *v_off = nullptr;     // pair ids of each such box (CSR)
  int32_t *v_pair = nullptr;
  int nvbox = 0;
  int64_t nvpair = 0;
  // per level: non-leaf boxes, CSR of their children (for the M2M sums)
  std::vector<int32_t *> m2m_tgt, m2m_off, m2m_kid;
  std::vector<int> m2m_n;
};

// Device buffers of a tree (sorted order, boxes, lists, leaf items) that
// plans on the same points share; freed when the last plan holding them is.
struct SharedAllocs {
  std::vector<void *> ptrs;
  ~SharedAllocs() {
    for (void *p : ptrs) (void)hipFree(p);
  }
};

}  // namespace fmm

struct fmm_plan {
  int kernel = 0, p = 0, ncrit = 0, precision = 0;
  double kappa = 0;
  int64_t n = 0;
  int nsurf = 0, ld = 0;           // surface points, padded leading dimension
  double lo[3] = {0, 0, 0}, W = 1, shift[3] = {0, 0, 0};
  int device = 0;
  // host tree
  std::vector<int64_t> keys, perm;
  std::vector<int32_t> level, nchild;
  std::vector<int64_t> anchor, begin, end, parent, child_begin;
  std::vector<int64_t> level_begin;  // size maxlevel+2
  std::vector<int32_t> mol;          // molecule of each box
  std::vector<int64_t> mol_off;      // point ranges of the molecules (input order)
  std::vector<double> mol_lo;        // lower corner of each molecule's root cube
  std::vector<int64_t> loff[4];      // U, V, W, X CSR offsets (nbox+1)
  std::vector<int64_t> lidx[4];
  std::vector<int32_t> leaf_ids;
  std::vector<int32_t> vpair_src, vpair_tgt;  // V pairs in GEMM order
  std::vector<int32_t> p2l_boxes;             // boxes whose X list goes through P2L
  int64_t p2p_inter = 0, far_inter = 0;
  std::vector<int64_t> item_pairs;  // pair interactions (targets x near sources) per leaf item, in launch order
  // device
  fmm::DevTree dt;
  void *surf = nullptr;            // T4 grid offsets in [-1,1]^3, nsurf entries
  void *pool1 = nullptr;           // swizzled ld x ld matrices
  int64_t pool1_count = 0, poolbf_count = 0;
  void *pool_bf = nullptr;         // bf16x3 mode: split M2L operators
  int bf_kb = 0;                   // 32-wide k blocks per row block in pool_bf
  // matrix ids (pool1 unless noted) per level; -1 when absent
  std::vector<int> utu_id, vsu_id, utd_id, vsd_id;  // truncated-SVD factors
  std::vector<int> rank_u, rank_d;                  // their ranks
  std::vector<std::vector<int>> m2m_id;             // [parent level][octant]
  std::vector<std::vector<int>> l2l_id;             // [parent level][octant]
  std::vector<std::vector<int>> m2l_id;             // [level][343 offset code] (factored: the left factor L)
  std::vector<std::vector<int>> m2l_r_id;           // factored M2L: the right factor R, same indexing
  std::vector<std::vector<int>> m2l_k;              // factored M2L: rank k per (level, offset)
  int m2l_ldt = 0;                                  // factored M2L: row length of the per-pair intermediate
  std::vector<double> vs_alpha, k_alpha;            // Laplace level scaling
  // work arrays, sized for work_nr columns
  int work_nr = 0;
  void *qs = nullptr, *equ = nullptr, *chk = nullptr, *eqd = nullptr, *chku = nullptr,
       *cu = nullptr, *yd = nullptr, *pairbuf = nullptr, *mslot = nullptr, *ydx = nullptr, *m2l_t = nullptr;
  // cu: upward check in singular coordinates (U_u^T chk); yd: downward
  // check in singular coordinates (M2L sums + U_d^T chk)
  fmm::PassLists lists_by_nr[fmm::MAX_NR + 1];  // task lists per column count
  // P2M targets (leaves at level >= 2) and per-leaf flags
  int p2m_count = 0;
  int32_t *d_p2m_box = nullptr;   // box ids
  int32_t *d_p2m_off = nullptr;   // 0..p2m_count (each box is its own source)
  int32_t *d_has_local = nullptr; // per leaf slot: level >= 2
  int32_t *d_m2l_rows = nullptr;  // per box: rows of its M2L sums (its level's downward rank, to 16)
  // profiling: event pairs per phase, recorded during fmm_eval
  int profiling = 0;               // bit k set: time phase k
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_events;
  std::vector<hipEvent_t> event_pool;
  // pair evaluation (this plan as the Laplace half): side stream, fork and
  // join events, and the near-field running sums of both kernels
  // the device's shared side streams: far passes; early near items; early M2L levels
  hipStream_t aux = nullptr, aux2 = nullptr, aux3 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_up = nullptr, ev_m2l = nullptr, ev_near = nullptr;
  hipEvent_t ev_m2m = nullptr, ev_m2lf = nullptr;  // the first M2M level done; the early M2L levels done
  void *pair_acc = nullptr;
  size_t pair_acc_bytes = 0;
  void *dips = nullptr;             // monopole + dipole sources: dipole records in Morton order
  // chained launches of a pair evaluation led by this plan: the M2M levels
  // and the L2L levels of both plans, each in one launch; counters (ticket,
  // finished tasks per phase, error flag) cleared before each launch
  fmm::Chain chain_up, chain_down;
  int32_t *chain_ctr = nullptr;
  int chain_ctr_n = 0;
  uint64_t coord_hash = 0;          // checksum of the FP64 input coordinates (per molecule, chained)
  uint64_t tree_hash = 0;           // fingerprint of coordinates, points, boxes and leaf items
  void *adj = nullptr;              // adjoint scratch: psi and grad psi
  size_t adj_bytes = 0;
  int64_t device_bytes = 0;
  double setup_ms = 0;
  double setup_split[5] = {0, 0, 0, 0, 0};  // sort, tree, lists, items, operators (ms)
  int tree_on_device = 0, tree_shared = 0;
  fmm_tuning_t tune{32, 16, 512, 16384, 1.15, 0, 0, 4, 0, 512, 0, 64, 0, 0, 1024, 0, 0};  // tunables in force at setup
  std::vector<void *> allocs;      // everything to free
  std::shared_ptr<fmm::SharedAllocs> tree_mem;  // the tree's device buffers (shared with plans on the same points)
  std::shared_ptr<fmm::SharedAllocs> ops_mem;   // translation operators (shared with plans of the same kernel on the same tree)
  int ops_shared = 0;
  std::vector<void *> *alloc_sink = nullptr;    // where dev_alloc records a buffer (null: allocs)
};

/*
 * fmmbem.h -- C ABI of the MI355X FMM-BEM library (libfmmbem.so).
 *
 * The library evaluates, on one AMD Instinct MI355X (gfx950), the
 * FMM-accelerated boundary-element matrix-vector product that dominates the
 * GMRES solve of the paper's Bempp-Exafmm linearised Poisson-Boltzmann
 * solver (Wang, Cooper, Betcke, Barba, arXiv 2103.01048; Methods,
 * "FMM-accelerated evaluation of integral operators" and "Fast multipole
 * method").
 *
 * Conventions shared by every entry point
 *   - Lengths in Angstrom, charges in e.  Kernels (Methods, boundary integral
 *     formulation): Laplace g = 1/(4 pi r), Yukawa g = exp(-kappa r)/(4 pi r).
 *   - "gradient" is +grad_x of the potential at the target (not the field).
 *   - A pair of points at zero distance (bitwise-equal coordinates)
 *     contributes nothing.  Bitwise-equal points always share a leaf (equal
 *     Morton keys).  Single precision (FMM_FP32, FMM_FP32_BF16X3) stores each
 *     point relative to the centre of its leaf, so two DISTINCT points in
 *     different leaves must be more than about 2^-21 of their leaf's width
 *     apart (1e-7 A for leaves of 0.5 A); closer pairs may round to zero
 *     separation and give non-finite results.  FMM_FP64 resolves them.
 *   - Device pointers are HIP device allocations owned by the caller; the
 *     library never frees them.  Plans and operators own their internal
 *     buffers and release them in *_free.
 *   - Every call that takes a stream enqueues its work on that stream and
 *     returns without synchronising, except fmm_setup and bem_setup, which
 *     synchronise the stream once.  A null stream is the default stream.
 *   - No exception crosses the ABI.  Every int-returning call returns one of
 *     the FMM_* status codes; fmm_last_error() gives a message for the last
 *     failure on the calling thread.
 *   - A plan or operator may be used by one stream at a time: evaluations
 *     share its workspace.
 */
#ifndef FMMBEM_H
#define FMMBEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_plan fmm_plan;
typedef struct bem_op bem_op;
typedef void *fmm_stream_t; /* a hipStream_t */

enum { FMM_LAPLACE = 0, FMM_YUKAWA = 1 };

/* Arithmetic of the evaluation.
 *   FMM_FP64        every stage in double precision (P2P on FP64 VALU,
 *                   translations on FP64 MFMA)
 *   FMM_FP32        single precision; translations on FP32 MFMA
 *   FMM_FP32_BF16X3 single precision; the M2L translations (the largest
 *                   dense contraction) on bf16 MFMA with each FP32 operand
 *                   split into a bf16 high and low part (three products,
 *                   FP32 accumulation), the other translations on FP32 MFMA
 * Densities, potentials and gradients are double for FMM_FP64, float
 * otherwise. */
enum { FMM_FP64 = 0, FMM_FP32 = 1, FMM_FP32_BF16X3 = 2 };

enum {
  FMM_OK = 0,
  FMM_EINVAL = -1,     /* bad argument */
  FMM_ENOMEM = -2,     /* device or host allocation failed */
  FMM_EHIP = -3,       /* a HIP runtime call failed */
  FMM_ENOTCONV = -4,   /* GMRES hit maxiter before the tolerance */
  FMM_EBREAKDOWN = -5  /* GMRES breakdown (non-finite residual) */
};

/* ------------------------------------------------------------------------
 * Fast multipole evaluation of the particle sum
 *      pot_i = sum_{j != i} g(|x_i - x_j|) q_j,   grad_i = grad_x pot_i
 * with targets = sources = the n points (the N-body sum of "FMM-accelerated
 * evaluation of integral operators").  Kernel-independent FMM ("Fast
 * multipole method"): an adaptive octree that splits a box while it holds
 * more than ncrit points; upward and downward equivalent densities on cube
 * surfaces of p x p x p grid points (n_surf = 6 (p-1)^2 + 2 points); P2M,
 * M2M, M2L, L2L, L2P and P2P in the paper's pass order.
 * ------------------------------------------------------------------------ */

/* Build a plan for the points xyz_dev (device, n x 3 doubles, row-major,
 * read during the call only).  kernel: FMM_LAPLACE or FMM_YUKAWA; kappa >= 0
 * (used by Yukawa only); p in [2, 10] (the paper's runs use p = 3 ... 10;
 * the surface kernels keep one surface point per thread of a workgroup of
 * at most 512 threads, n_surf = 488 at p = 10); ncrit >= 1; precision: FMM_FP64,
 * FMM_FP32 or FMM_FP32_BF16X3.  Sorts the points along a Morton curve on the
 * device, builds the tree and interaction lists on the host, precomputes the
 * translation operators in FP64 (truncated-SVD pseudo-inverses of the
 * check-to-equivalent kernel matrices) and uploads them.  Synchronises
 * `stream` once.  n = 0 gives a valid empty plan.  Errors: FMM_EINVAL for
 * n < 0, a null output, a non-finite coordinate, p or ncrit out of range,
 * kappa < 0 or non-finite; FMM_ENOMEM; FMM_EHIP. */
int fmm_setup(const double *xyz_dev, int64_t n, int kernel, double kappa, int p, int ncrit,
              int precision, fmm_stream_t stream, fmm_plan **out);

/* Plan for a batch of nmol independent point sets ("molecules"): molecule m
 * is points offsets[m] .. offsets[m+1]-1 of xyz_dev (offsets: HOST array of
 * nmol+1 nondecreasing values, offsets[0] = 0).  Points of different
 * molecules do not interact.  Every molecule gets its own root cube, all of
 * the same side (the largest extent in the batch), so that the translation
 * operators are shared and each FMM pass runs as one launch for the whole
 * batch.  fmm_eval on such a plan evaluates every molecule; densities and
 * outputs use the concatenated order.  Otherwise as fmm_setup. */
int fmm_setup_batch(const double *xyz_dev, const int64_t *offsets, int nmol, int kernel, double kappa, int p,
                    int ncrit, int precision, fmm_stream_t stream, fmm_plan **out);

/* Evaluate nrhs density columns.  q_dev: nrhs x n (column c at q_dev + c*n),
 * in the caller's point order, element type double (FMM_FP64) or float.
 * pot_dev: nrhs x n, same type; grad_dev: nrhs x n x 3 (gradient of point i
 * of column c at grad_dev + (c*n + i)*3), or NULL to skip gradients.
 * 1 <= nrhs <= 64.  Asynchronous on `stream`.  Errors: FMM_EINVAL for a null
 * plan or buffer, nrhs out of range; FMM_ENOMEM when the workspace for a
 * larger nrhs cannot be allocated; FMM_EHIP for a failed launch. */
int fmm_eval(fmm_plan *plan, const void *q_dev, int nrhs, void *pot_dev, void *grad_dev,
             fmm_stream_t stream);

/* Evaluate two plans on the same densities: the Laplace and the Yukawa
 * potentials that the direct formulation's operators need for one input
 * (Methods, eq:direct and eq:bempp_fmm_matvec).  Results are those of
 * fmm_eval(plan_a, ...) and fmm_eval(plan_b, ...), with the same layouts;
 * grad_a_dev / grad_b_dev may be NULL.  When plan_a is a Laplace plan and
 * plan_b a Yukawa plan built from the same points (and batch offsets) with
 * the same p, ncrit and precision, the two share one tree: the far-field
 * passes of both kernels run as shared launches on an internal stream
 * while the near field of both kernels runs on `stream` in one launch that
 * computes each pair distance once; otherwise the two evaluations run one
 * after the other on `stream`.  The internal streams (three, default priority)
 * belong to the device, not to the plans: every pair evaluation on a device
 * uses the same three, so the hardware queues taken do not grow with the number
 * of plans, pair evaluations issued from different caller streams at once
 * queue their side passes one after the other, and a pair evaluation must not
 * be captured into a graph while another thread evaluates a pair on the same
 * device.  They live until the process ends.  Asynchronous on `stream` (the
 * internal streams are joined back into it).  Errors: as fmm_eval; FMM_EINVAL
 * when the plans differ in point count or precision. */
int fmm_eval_pair(fmm_plan *plan_a, fmm_plan *plan_b, const void *q_dev, int nrhs, void *pot_a_dev,
                  void *grad_a_dev, void *pot_b_dev, void *grad_b_dev, fmm_stream_t stream);

/* Potentials of monopole and dipole sources (one column, no gradients) for a
 * Laplace plan_a and a Yukawa plan_b sharing one tree (same points, batch
 * offsets, p, ncrit and precision; FMM_EINVAL otherwise):
 *   pot_k(x_i) = sum_{j: r_ij > 0} [ qscale_k q_j g_k(r_ij) + dip_j . grad_y g_k(x_i, y_j) ]
 * with grad_y g = +(x - y) (1 + kappa r) e^{-kappa r} / (4 pi r^3) (kappa = 0
 * for Laplace).  This is the double-layer plus single-layer potential of the
 * direct formulation in one pass per kernel (Methods, eq:single_double and
 * eq:direct: the double layer is the normal derivative of g at the source).
 * q_dev: n charges; dip_dev: n x 3 dipole moments (row i = point i); pot_a_dev,
 * pot_b_dev: n each; grad_a_dev, grad_b_dev: n x 3 gradients +grad_x pot_k
 * (the hypersingular and adjoint double-layer terms of the derivative
 * formulation, eq:juffer and eq:adj_hyp, come from their normal
 * components), or both NULL for potentials only; caller's point order;
 * element type double for FMM_FP64, float otherwise.  Equivalent densities
 * stay monopoles, so only the source side (P2M, P2L, near field) differs
 * from fmm_eval_pair.  Asynchronous on `stream` (internal side stream joined
 * back).  Errors: FMM_EINVAL for null buffers, non-finite scales or plans
 * that do not share a tree. */
int fmm_eval_pair_md(fmm_plan *plan_a, fmm_plan *plan_b, const void *q_dev, const void *dip_dev, double qscale_a,
                     double qscale_b, void *pot_a_dev, void *grad_a_dev, void *pot_b_dev, void *grad_b_dev,
                     fmm_stream_t stream);

/* Adjoint of fmm_eval for a loss L(pot) with upstream gradient gbar_dev =
 * dL/dpot (nrhs x n, same type and layout as pot).  Because the kernel is
 * symmetric and targets = sources, the density gradient is one more
 * evaluation, dq = G gbar; the position gradient of point k (summed over the
 * columns) is  dxyz_k = sum_c [gbar_ck grad(pot_c)_k + q_ck grad(psi_c)_k]
 * with psi = G gbar.  q_dev and grad_fwd_dev are the forward densities and
 * the forward gradient output (nrhs x n x 3).  dq_dev (nrhs x n) and
 * dxyz_dev (n x 3) are written; either may be NULL to skip it.  Gradients
 * of L with respect to the forward gradient output are not supported (they
 * need second derivatives of the kernel).  Asynchronous. */
int fmm_adjoint(fmm_plan *plan, const void *q_dev, const void *gbar_dev, const void *grad_fwd_dev, int nrhs,
                void *dq_dev, void *dxyz_dev, fmm_stream_t stream);

/* Tunable parameters of the plans set up afterwards (process-wide; each plan
 * keeps the values it was set up with).  The defaults are the values below;
 * paper_2103_01048_amd.autotune picks them, with ncrit, per expansion order
 * and point count on the device at hand.
 *   tile_split2   a leaf tile of at most this many targets (<= 32) runs as
 *                 2 half-waves that take the sources in turn (32; 0: never)
 *   tile_split4   ... of at most this many (<= 16) as 4 quarter-waves (16; 0: never)
 *   work_cap_min, work_cap_div
 *                 a leaf tile whose source work exceeds
 *                 max(work_cap_min, total work / work_cap_div) point-source
 *                 evaluations is cut into parts of about that size (512, 16384)
 *   far_weight    work of one surface source relative to a point source when
 *                 items are cut and ordered (1.15)
 *   gemm_rbw      16-row blocks per wave in the single-precision translation
 *                 GEMMs (0: automatic, 1 .. 8)
 *   m2l_factored  1: each M2L operator (per level and offset, in the
 *                 truncated-SVD coordinates) is split by its own truncated
 *                 SVD, M ~ L R with rank k (singular values above 1e-7 of the
 *                 largest in single precision, 1e-11 in FP64), and applied in
 *                 two gather-GEMM passes (R to a k-value intermediate per
 *                 pair, then L); 0: one dense pass (the default)
 *   pair_order    pair evaluations, the caller's stream (the far-field
 *                 passes run on a side stream meanwhile): 0 near field once
 *                 P2M is done, then P2L; 1 P2L once P2M is done, near field
 *                 once the upward pass is done; 2 P2L, then the near field,
 *                 both once P2M is done; 3 P2L, its projection
 *                 and the M2P sources' equivalent densities once P2M is done
 *                 (beside the upward GEMMs and the M2L), the near field once
 *                 the M2L is done (beside the M2L sums and the downward pass);
 *                 4 (the default) the same overlap with the roles of the
 *                 streams swapped:
 *                 P2M, the upward GEMMs, the M2L and then the near field on
 *                 the caller's stream (no wait across streams on that path),
 *                 P2L and the downward pass on the side stream
 *   near_lds      pair evaluations: LDS bytes (0..65536, unused by the
 *                 kernel) reserved per near-field wave, which caps the
 *                 near-field waves per compute unit so that the far-field
 *                 passes on the side stream find room beside them; 0: none
 *   gemm_lat      translation GEMM launches of at most this many workgroups
 *                 (0..1<<20) run the latency-bound form (all operands of a
 *                 workgroup fetched at once); 0: never; default 512
 *   gemm_chain    pair evaluations: 1 runs the M2M levels of both plans in
 *                 one launch and the L2L levels in another (tasks in
 *                 dependency order, each level waiting on counters of the
 *                 one before, bounded waits); 0: one launch per level
 *   m2l_cols      bf16x3 M2L columns (V pairs) per workgroup sharing one
 *                 operator fetch: 64 (default) or 128
 *   gemm_narrow   pair evaluations in single precision: 1 runs the L2L and
 *                 the leaves' downward projections as one-wave workgroups
 *                 (room beside the near field's waves); 0: 256-thread ones
 *   near_early, near_early_grid
 *                 pair evaluations with pair_order 3 or 4: the last near_early
 *                 per mille (0..900) of the near-field items (the shortest)
 *                 start at once on a second side stream, on a grid of
 *                 near_early_grid waves (64..65536) that loop over them,
 *                 beside the upward passes and the M2L; 0: none
 *   near_early_start
 *                 with near_early: 0 starts the early items with the
 *                 far-field passes, 1 once P2M (VALU work on the path of
 *                 the upward pass) is done
 *   m2l_early     pair evaluations: 1 runs the M2L of the two finest levels
 *                 on a third side stream as soon as their upward densities
 *                 are final (after the first M2M level), beside the coarser
 *                 M2M levels, and the rest of the M2L after them; 0: one
 *                 M2L launch after the upward pass (default)
 * FMM_EINVAL for values out of range. */
typedef struct {
  int32_t tile_split2;
  int32_t tile_split4;
  int32_t work_cap_min;
  int32_t work_cap_div;
  double far_weight;
  int32_t gemm_rbw;
  int32_t m2l_factored;
  int32_t pair_order;
  int32_t near_lds;
  int32_t gemm_lat;
  int32_t gemm_chain;
  int32_t m2l_cols;
  int32_t gemm_narrow;
  int32_t near_early;
  int32_t near_early_grid;
  int32_t m2l_early;
  int32_t near_early_start;
} fmm_tuning_t;
int fmm_set_tuning(const fmm_tuning_t *tuning);
int fmm_get_tuning(fmm_tuning_t *tuning);

/* Sizes of the plan's tree, for tests and reports. */
typedef struct {
  int64_t n_points;
  int64_t n_boxes;
  int64_t n_leaves;
  int32_t max_level;
  int32_t n_surf;        /* points per equivalent/check surface */
  int64_t n_u_pairs;     /* leaf-leaf near-field pairs (U lists) */
  int64_t n_v_pairs;     /* M2L pairs (V lists) */
  int64_t n_w_pairs;     /* M2P pairs (W lists) */
  int64_t n_x_pairs;     /* P2L pairs (X lists) */
  int64_t n_p2p_interactions; /* sum over leaves of targets x U-list sources */
  int64_t device_bytes;  /* device memory held by the plan */
  double setup_ms;       /* wall time of fmm_setup */
  int64_t n_far_interactions; /* leaf targets x surface points (M2P + L2P) */
  int32_t rank_up;       /* kept singular values of the upward check-to-equivalent map (max over levels) */
  int32_t rank_down;     /* same, downward */
  /* wall time of the stages of fmm_setup, milliseconds */
  double setup_sort_ms;  /* bounding box, Morton keys, radix sort on the device, sorted keys to the host */
  double setup_tree_ms;  /* octree levels */
  double setup_lists_ms; /* U, V, W, X lists */
  double setup_items_ms; /* points into leaf order, leaf work items, near and far ranges, upload */
  double setup_ops_ms;   /* translation operators (FP64 truncated SVDs and products), upload */
  int32_t tree_on_device; /* 1: octree and lists built by device kernels */
  int32_t tree_shared;    /* 1: tree, lists and leaf items taken from a live plan on the same points */
  int32_t chain_timeouts; /* nonzero: a wait of a chained launch (gemm_chain) led by this plan hit its
                             bound, and the evaluation it belonged to is not valid (never expected:
                             the chain drains by construction; fmm_info synchronises to read it) */
  int64_t n_p2p_early;    /* of n_p2p_interactions, those in the near-field items that a pair
                             evaluation led by this plan starts early (tunable near_early); the
                             rest run in the main near-field launch */
  int32_t n_items;        /* leaf work items: waves of the near- and far-field launches */
  int32_t n_items_early;  /* of those, the items started early (the early launch loops over them) */
} fmm_info_t;

int fmm_info(const fmm_plan *plan, fmm_info_t *out);

/* Copy the plan's tree to host arrays (test access to the integer work).
 * Any pointer may be NULL to skip that array.
 *   perm   [n_points]   sorted position -> caller index (int64)
 *   keys   [n_points]   sorted 63-bit Morton keys (int64)
 *   level, anchor_xyz (3 per box), begin, end, parent, child_begin, nchild
 *          [n_boxes]    boxes ordered by (level, key)
 *   list_off [4*(n_boxes+1)], list_idx [n_u+n_v+n_w+n_x]: the U, V, W, X
 *          lists in CSR form, one after the other (list k of box b is
 *          list_idx[list_off[k*(nb+1)+b] .. list_off[k*(nb+1)+b+1]),
 *          offsets counted from the start of list_idx), each sorted. */
int fmm_get_tree(const fmm_plan *plan, int64_t *perm, int64_t *keys, int32_t *level,
                 int64_t *anchor_xyz, int64_t *begin, int64_t *end, int64_t *parent,
                 int64_t *child_begin, int32_t *nchild, int64_t *list_off, int64_t *list_idx);

/* Root cube of the plan: lower corner (3 doubles) and side. */
int fmm_get_root(const fmm_plan *plan, double *lo3, double *width);

/* Per-phase timing with HIP events recorded on the evaluation stream.
 * fmm_set_profiling(plan, mask) makes later fmm_eval calls record an event
 * pair around every launch group of each phase k with bit k set in `mask`
 * (0 switches timing off, FMM_PHASE_ALL times every phase; each event pair
 * costs a few microseconds of stream time); fmm_get_phase_times synchronises
 * on those events,
 * writes the accumulated milliseconds and launch counts of the first
 * `nphase` phases (FMM_PHASE_COUNT at most) and clears them. */
enum {
  FMM_PHASE_PERMUTE = 0, /* densities into Morton order */
  FMM_PHASE_P2M = 1,     /* leaf sources -> upward check potentials */
  FMM_PHASE_UC2E = 2,    /* upward check -> equivalent (MFMA) */
  FMM_PHASE_M2M = 3,     /* children -> parent upward densities (MFMA) */
  FMM_PHASE_P2L = 4,     /* X-list sources -> downward check potentials */
  FMM_PHASE_M2L = 5,     /* V-list translations (MFMA) */
  FMM_PHASE_M2L_SUM = 6, /* per-box sum of the M2L pair results */
  FMM_PHASE_L2L = 7,     /* parent downward density -> child check (MFMA) */
  FMM_PHASE_DC2E = 8,    /* downward check -> equivalent (MFMA) */
  FMM_PHASE_LEAF = 9,    /* P2P + M2P + L2P at the leaves, unpermute, 1/(4 pi) */
  FMM_PHASE_NEAR = 10,   /* fmm_eval_pair: P2P of both kernels (first plan's timer) */
  FMM_PHASE_FAR = 11,    /* fmm_eval_pair: M2P + L2P of both kernels, unpermute */
  FMM_PHASE_NEAR_EARLY = 12, /* fmm_eval_pair: the near-field items started early (near_early) */
  FMM_PHASE_COUNT = 13,
  FMM_PHASE_ALL = 0x1fff,
  /* flag in the fmm_set_profiling mask: pair evaluations led by this plan
   * run every pass on the caller's stream, one after the other (no side
   * stream), so that each phase's time is its own and not stretched by the
   * passes that otherwise share the GPU with it; for measurement only */
  FMM_PROFILE_SERIAL = 0x10000
};
int fmm_set_profiling(fmm_plan *plan, int enable);
int fmm_get_phase_times(fmm_plan *plan, double *ms, int64_t *launches, int nphase);

/* Release a plan and its device buffers (NULL is a no-op).  Waits for the
 * device's side streams if the plan led a pair evaluation (they may also hold
 * other plans' queued work) and for any evaluation of the plan still queued;
 * the side streams themselves stay for the process. */
void fmm_free(fmm_plan *plan);

/* ------------------------------------------------------------------------
 * Boundary-element operators (Methods, boundary integral formulation) for
 * the solute-side potential u and its normal derivative v on the molecular
 * surface, with piecewise-constant (P0) Galerkin discretisation on a
 * triangle mesh and the matrix-vector split A x = P2^T (G - C) P1 x + S x
 * ("FMM-accelerated evaluation of integral operators").  Two formulations:
 *
 * FMM_BEM_DIRECT (eq:direct, Yoon-Lenhoff):
 *   [ M/2 + K_L    -V_L            ] [u]   [b]
 *   [ M/2 - K_Y    (eps1/eps2) V_Y ] [v] = [0],     M = diag(triangle areas)
 *
 * FMM_BEM_DERIVATIVE (eq:juffer, Juffer et al.), e21 = eps2/eps1, e12 = eps1/eps2:
 *   [ (1 + e21)/2 M - (e21 K_Y - K_L)   V_Y - V_L                        ] [u]   [b ]
 *   [ W_Y - W_L                         (1 + e12)/2 M + e12 K'_Y - K'_L  ] [v] = [b'],
 *   b' the normal derivative of the Coulomb term; K' the adjoint double
 *   layer and W the hypersingular operator (eq:adj_hyp).  Only the
 *   difference W_Y - W_L appears; its kernel is weakly singular.
 *
 * FMM_BEM_EXTERIOR (eq:lu, the exterior variant of Lu and co-workers): the
 *   same equations scaled by e12 and solved for the solvent-side unknowns
 *   u = phi_2 and v = d phi_2/dn:
 *   [ (1 + e12)/2 M - (K_Y - e12 K_L)   V_Y - V_L                        ] [u]   [b ]
 *   [ e12 (W_Y - W_L)                   (1 + e12)/2 M + e12 K'_Y - K'_L  ] [v] = [b'],
 *   b and b' with 1/eps_out in place of 1/eps_in.
 *
 * FMM_BEM_EXTERIOR_P1: the exterior formulation on continuous piecewise-
 *   linear elements (Results: the exterior variant with P1 elements and
 *   mass-matrix preconditioning).  Unknowns per VERTEX (u = phi_2, v =
 *   d phi_2/dn at each vertex; vectors of 2*nv doubles, every vertex on a
 *   triangle); the hat function of a vertex is the barycentric coordinate of
 *   its corner on each triangle.  Quadrature-point densities interpolate the
 *   vertex values; test integrals weight by the hat functions and are added
 *   per vertex in a fixed order; M is the P1 mass matrix (A/12 (1 + delta_ab)
 *   per triangle); the S - C corrections are 3 x 3 blocks per pair with the
 *   Laplace inner integral of a linear density in closed form.  Only the
 *   lumped mass preconditioner (FMM_BEM_PRECOND_MASS) applies.
 *
 * V and K are the single- and double-layer operators of the Laplace (L) and
 * Yukawa (Y) kernels.  G is evaluated by one fmm_eval_pair_md call per
 * product (charges W v and dipoles W u n at the regular quadrature points;
 * the derivative formulation also takes the gradients).  For pairs of
 * triangles that share a vertex the regular-rule values C are replaced by
 * accurate values S (closed-form inner integrals of the Laplace part over
 * the flat triangle, Gauss rules for the bounded or weakly singular
 * Yukawa-minus-Laplace remainders; K' uses the transposed K pair), applied
 * as one precomputed sparse FP64 matrix S - C.
 * ------------------------------------------------------------------------ */
enum { FMM_BEM_DIRECT = 0, FMM_BEM_DERIVATIVE = 1, FMM_BEM_EXTERIOR = 2, FMM_BEM_EXTERIOR_P1 = 3 };
/* Preconditioners (Results, the preconditioners of the two formulation
 * families): per-triangle 2 x 2 block-diagonal (the inverse of A's block on
 * the identical pair, after Altman and co-workers; P0 only) or the mass
 * matrix diag(M, M) (diagonal for P0 elements, so mass lumping is exact; for
 * P1 elements its lumped form, per vertex the sum of area/3 over its
 * triangles). */
enum { FMM_BEM_PRECOND_BLOCK = 0, FMM_BEM_PRECOND_MASS = 1 };

/* Build the operator.  verts (nv x 3 doubles) and tris (nt x 3 int32, vertex
 * indices, counter-clockwise seen from the solvent so that normals point
 * out of the molecule) are HOST arrays read during the call.  quad_pts: 3 or
 * 6 (regular rule per triangle); eps_in, eps_out > 0; kappa >= 0; p, ncrit,
 * precision as for fmm_setup (the two FMM plans); formulation:
 * FMM_BEM_DIRECT, FMM_BEM_DERIVATIVE, FMM_BEM_EXTERIOR or FMM_BEM_EXTERIOR_P1.
 * The preconditioner starts as FMM_BEM_PRECOND_BLOCK (FMM_BEM_PRECOND_MASS
 * for P1).  Synchronises `stream`.  Errors:
 * FMM_EINVAL for bad sizes, indices or parameters, a degenerate triangle;
 * FMM_ENOMEM; FMM_EHIP. */
int bem_setup(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, int quad_pts, double eps_in,
              double eps_out, double kappa, int p, int ncrit, int precision, int formulation, fmm_stream_t stream,
              bem_op **out);

/* y = A x; x_dev, y_dev: device, 2*n doubles ([u; v] and the two row
 * blocks; n = nt, or nv for P1 elements: bem_info's n_unknowns).  x_dev and y_dev must not overlap.  Asynchronous. */
int bem_matvec(bem_op *op, const double *x_dev, double *y_dev, fmm_stream_t stream);

/* Right-hand side b_dev (2*n doubles) for nq point charges at qxyz_dev
 * (device, nq x 3) with charges q_dev (device, nq), e and Angstrom:
 * b_s = int_Ts (1/eps) sum_k q_k / (4 pi |x - r_k|), eps = eps_out for the
 * exterior formulations (P0 and P1) and eps_in otherwise; second block 0
 * (direct) or int_Ts n_s . grad of the same sum (derivative, exterior); P1:
 * the same fields tested with the hat functions, b_i summed over the
 * triangles at vertex i; regular rule, FP64 direct sums.  Asynchronous. */
int bem_rhs(bem_op *op, const double *qxyz_dev, const double *q_dev, int64_t nq, double *b_dev,
            fmm_stream_t stream);

/* bem_rhs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * same launches as bem_rhs (bitwise equal result) with no allocation and no
 * free: its two temporary arrays (nq scaled charges, rounded up to 32, then
 * the field at the operator's n_points quadrature points) live in one static
 * device array of BEM_RHS_SCRATCH_DOUBLES doubles (64 MiB) per GPU, which the
 * library holds until the process ends.  Requires
 * roundup32(max(nq, 1)) + n_points <= BEM_RHS_SCRATCH_DOUBLES (bem_info's
 * n_points), FMM_EINVAL otherwise, before any launch.  Every call on one GPU
 * uses that GPU's array: calls that overlap in time on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 * Asynchronous on `stream`; other errors as bem_rhs. */
#define BEM_RHS_SCRATCH_DOUBLES (1 << 23)
int bem_rhs_noalloc(bem_op *op, const double *qxyz_dev, const double *q_dev, int64_t nq, double *b_dev,
                    fmm_stream_t stream);

/* Polar solvation energy (kcal/mol) of the charges for the solution x_dev of
 * the operator's formulation (exterior unknowns are first mapped to the
 * solute side, v -> (eps_out/eps_in) v, by the interface conditions):
 * reaction potential phi_reac(r_k) = -K_L u + V_L v evaluated at the charges
 * (eq. of the reaction potential, FP64 direct sum over the quadrature
 * points; P1 vertex values interpolated to them), dG = 1/2 sum_k q_k phi_reac(r_k) * 4 pi * 332.0637 (FP64
 * reduction on the device).  Synchronises `stream`; result in *dG. */
int bem_energy(bem_op *op, const double *x_dev, const double *qxyz_dev, const double *q_dev, int64_t nq,
               double *dG, fmm_stream_t stream);

/* Select the preconditioner used by bem_precondition and gmres_solve:
 * FMM_BEM_PRECOND_BLOCK or FMM_BEM_PRECOND_MASS (FMM_EINVAL otherwise, and
 * for BLOCK on P1 elements).
 * Asynchronous on `stream`. */
int bem_set_preconditioner(bem_op *op, int kind, fmm_stream_t stream);

/* Apply the selected preconditioner (per triangle a 2 x 2 block: the inverse
 * of A's block on the identical pair, or diag(1/area, 1/area); P1: per
 * vertex 1 / its lumped mass): y = P^-1 x.  Device vectors of 2*n doubles.
 * Asynchronous. */
int bem_precondition(bem_op *op, const double *x_dev, double *y_dev, fmm_stream_t stream);

/* FP64 GMRES on A x = b with right preconditioning (bem_precondition),
 * classical Gram-Schmidt with reorthogonalisation on the device and Givens
 * rotations on the host.  restart: Krylov dimension before a restart
 * (<= 0: maxiter, full GMRES).  Stops when the recomputed residual
 * |b - A x| / |b| <= tol.  x_dev holds the initial guess and receives the
 * solution.  refine (may be NULL): an operator other than op on the same
 * mesh with the same formulation, quadrature rule, permittivities and kappa
 * (FMM_EINVAL otherwise), usually FMM_FP64 with a higher order; then the
 * solve is an iterative refinement:
 * residuals are computed with `refine` and each correction is solved with
 * `op` to a relative tolerance inner_tol.  iters (may be NULL) receives the
 * total number of inner iterations; resid_hist (host, may be NULL, maxiter
 * entries) the estimated relative residual after each inner iteration.
 * Synchronises `stream` every iteration.  Returns FMM_OK, FMM_ENOTCONV
 * (maxiter reached; x holds the last iterate) or FMM_EBREAKDOWN. */
int gmres_solve(bem_op *op, bem_op *refine, const double *b_dev, double *x_dev, double tol, double inner_tol,
                int maxiter, int restart, int *iters, double *resid_hist, fmm_stream_t stream);

typedef struct {
  int64_t n_triangles;
  int64_t n_points;           /* quadrature points = FMM points */
  int64_t n_singular_pairs;   /* triangle pairs sharing a vertex (incl. identical) */
  int32_t quad_pts;
  int32_t precision;
  int32_t formulation;
  int32_t preconditioner;
  int64_t n_unknowns;         /* per block: nt (P0) or nv (P1); vectors hold 2x this */
} bem_info_t;
int bem_info(const bem_op *op, bem_info_t *out);

/* The FMM plan of kernel FMM_LAPLACE or FMM_YUKAWA used by the operator
 * (owned by the operator). */
fmm_plan *bem_fmm_plan(bem_op *op, int kernel);

void bem_free(bem_op *op);

/* Message of the last failed call on this thread ("" if none). */
const char *fmm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FMMBEM_H */

/*
 * vp.h -- C ABI of the MI355X volume-potential evaluation library (libvp.so).
 *
 * The library evaluates, on one AMD Instinct MI355X (gfx950), the
 * target-independent smooth quadrature of the volume potential
 *
 *     u_b(t_i) = sum_j G(r_j, t_i) w_j f_b(r_j)  +  sum_k C[i,k] f_b(r_k)
 *
 * with the 2D Laplace Green's function G(r, r0) = -(1/(2 pi)) log|r - r0|
 * (Section 2.1 of Anderson, Zhu and Veerapaneni, arXiv 2203.05933).  The first
 * sum is the smooth rule of Section 3.2 (eq. Tk_smooth_quad) whose "modified
 * weights" w_j = J^k(xi_j) w_j make it a plain point sum (Section 4.2 gives
 * the same rule for boxes), evaluated by a fast multipole method over an
 * adaptive quadtree.  The second is the sparse local correction matrix the
 * paper assembles from its per-cell maps Pi_k (Section 4, next to eqs.
 * ndofs/nsrcs).  A source/target pair at exactly zero distance (the self
 * pair when the targets are the nodes) contributes nothing to the first sum.
 *
 * Conventions
 *   * All floating-point arrays are float64, C-contiguous.  Batched arrays are
 *     [nbatch][len] (density b is the contiguous row b).
 *   * vp_plan takes HOST pointers and copies everything it needs into
 *     plan-owned device memory; the caller may free its arrays on return.
 *   * vp_eval* take DEVICE pointers owned by the caller (e.g. torch tensor
 *     data), in the caller's (user) order, never in the library's sorted
 *     order.  Outputs are overwritten, not accumulated.
 *   * Evaluations are asynchronous on the plan's stream; they do not
 *     allocate and do not synchronise the host.  Inputs must stay valid and
 *     unmodified until the stream reaches the evaluation.
 *   * A plan must not be used from two host threads at once.
 *   * No function throws or aborts: every error is a status code, with a
 *     message from vp_last_error.  VP_EINVAL leaves the plan usable.
 *     VP_EDEVICE (a HIP runtime error) poisons the plan: later calls on it
 *     return VP_EDEVICE.
 */
#ifndef VP_H
#define VP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vp_plan_s *vp_plan_t; /* opaque, library-owned */

typedef enum {
    VP_OK = 0,
    VP_EINVAL = 1,       /* invalid argument; nothing was done */
    VP_ENOMEM = 2,       /* device allocation failed */
    VP_EDEVICE = 3,      /* HIP runtime error; the plan is poisoned */
    VP_EUNSUPPORTED = 4, /* valid but outside what this build supports */
    VP_EINTERNAL = 5     /* internal limit exceeded (e.g. list traversal depth) */
} vp_status;

enum { VP_FP64 = 0, VP_FP32_BULK = 1 };
enum {
    VP_M2L_AUTO = 0,
    VP_M2L_FP64_MFMA = 1,   /* one real 2P x 2P operator per interaction offset, FP64 matrix cores */
    VP_M2L_FP32_MFMA = 2,   /* the same in FP32 (VP_FP32_BULK only) */
    VP_M2L_FP32_SPLIT = 3,  /* the same with hi/lo FP32 products (VP_FP32_BULK only) */
    VP_M2L_FP64_SCALED = 4, /* diagonally scaled form: complex scalings by powers of the
                               offset around one real P x P binomial matrix shared by all
                               offsets, FP64 matrix cores */
    VP_M2L_FP32_SCALED = 5  /* the scaled form in FP32 (VP_FP32_BULK only) */
};
enum { VP_P2P_AUTO = 0, VP_P2P_PAIRWISE = 1, VP_P2P_TABLES = 2 };
/* Green's function (Section 2.1):
   VP_KERNEL_LAPLACE: G(r, r0) = -(1/(2 pi)) log |r - r0|
   VP_KERNEL_YUKAWA:  G(r, r0) = (lambda^2 / (2 pi)) K_0(lambda |r - r0|), the
                      modified Helmholtz kernel of L = -Delta + lambda^2 in the
                      normalisation Section 2.1 writes (divide by lambda^2 for
                      the Green's function of -Delta + lambda^2 itself).  This
                      build evaluates it on uniform grids of congruent 64-point
                      leaves (targets = nodes, one leaf level, no W or X lists),
                      in float64, by fixed matrices per level: other trees,
                      VP_FP32_BULK and vp_eval_grad_targets return
                      VP_EUNSUPPORTED. */
enum { VP_KERNEL_LAPLACE = 0, VP_KERNEL_YUKAWA = 1 };
/* VP_FLAG_AUTOTUNE: with m2l_mode VP_M2L_AUTO, vp_plan tunes the evaluation
   by coordinate descent, timing full evaluations of this plan: the M2L kernel
   form (FP64: scaled and per-offset FP64 products; FP32-bulk: scaled FP32,
   per-offset FP32, split hi/lo FP32 and scaled FP64 products -- every one
   meets the precision's accuracy target), the waves per 16-column tile of the
   M2L and near-table kernels (4 or 2; a knob set in vp_options is kept), and
   three streams against one (kept on one stream with VP_FLAG_ONE_STREAM).
   Choices are cached per process for plans of the same geometry and options
   (a second such plan skips the timing).  vp_get_info reports them.
   VP_FLAG_AUTOTUNE_LEAF: also tune the tree shape -- vp_plan builds the plan
   with max_leaf and with max_leaf / 4 (when that is at least 4), each tuned as
   above, times them and keeps the faster (the leaf size enters the cache key's
   result).  Results differ only by rounding. */
/* VP_FLAG_ONE_STREAM: run every kernel of an evaluation on the plan's stream,
   in sequence.  By default the correction apply and the near field run on a
   second stream owned by the plan, beside the expansion passes, and join the
   plan's stream before the far field; with this flag nothing overlaps (for
   callers that need all work on one stream, and for per-stage timings
   without contention).  Results are identical either way. */
enum { VP_FLAG_AUTOTUNE = 1, VP_FLAG_ONE_STREAM = 2, VP_FLAG_AUTOTUNE_LEAF = 8 };

typedef struct {
    int32_t order;     /* p: highest power kept in the expansions (p+1 complex
                          coefficients including the log term); 1..60; default 30 */
    int32_t max_leaf;  /* a box is split while it holds more than max_leaf
                          sources or targets; 1..256; default 64 */
    int32_t nbatch;    /* densities per evaluation; 1..64; default 1 */
    int32_t precision; /* VP_FP64: every stage in float64.  VP_FP32_BULK: the
                          expansion stages (P2M, M2M, M2L, L2L, L2P, M2P, P2L)
                          in float32; charges, near field, translation
                          operator set-up and final accumulation in float64 */
    int32_t m2l_mode;  /* VP_M2L_*; AUTO = FP64_SCALED for VP_FP64,
                          FP32_SCALED for VP_FP32_BULK.  FP32_SPLIT forms
                          T_hi M_hi + T_hi M_lo + T_lo M_hi with FP32 MFMA */
    int32_t p2p_mode;  /* VP_P2P_*; AUTO uses precomputed near-field tables on
                          leaves whose nodes are congruent copies of one
                          pattern (uniform box grids) and the pairwise kernel
                          elsewhere */
    int32_t max_level; /* deepest tree level; 1..30; 0 = 30 */
    int32_t flags;     /* VP_FLAG_* bits; 0 = none */
    double root[3];    /* x0, y0, side of the root square; side <= 0 selects
                          the bounding square of sources and targets.  With
                          side > 0 every node and target must lie in the
                          closed square [x0, x0+side] x [y0, y0+side]
                          (VP_EINVAL otherwise) */
    void *stream;      /* hipStream_t for plan-time copies and evaluations;
                          NULL = the null stream */
    int32_t kernel;    /* VP_KERNEL_*; default VP_KERNEL_LAPLACE */
    int32_t m2l_waves; /* waves per 16-column tile of the M2L kernels: 2 or 4,
                          or 1 = one wave per tile, four tiles per workgroup
                          (scaled forms; the per-offset forms take 4);
                          0 = 1, or the autotuner's choice */
    double lambda;     /* VP_KERNEL_YUKAWA: lambda > 0 (Section 5 uses lambda^2 = 100) */
    int32_t table_waves; /* waves per 16-column tile of the near-table kernel:
                            2 or 4, or 1 = one wave over two tiles (each
                            operator fragment loaded once for both; patterns
                            of more than 64 points take 2 instead); 0 = 1, or
                            the autotuner's choice */
    int32_t reserved;
} vp_options;

/* Fill *opt with the defaults listed above. */
void vp_default_options(vp_options *opt);

/*
 * vp_plan -- build the static-geometry plan (the paper excludes this set-up
 * from its timings, Section 5 / Table 3).
 *   x, y, w [n]      : node coordinates and smooth-rule weights (host)
 *   tx, ty  [m]      : target coordinates (host), or both NULL: the targets
 *                      are the nodes (m must then equal n)
 *   rowptr [m+1], col [nnz], val [nnz] : correction matrix C in CSR form,
 *                      rows = targets, columns = nodes (host); rowptr NULL
 *                      means no correction.  rowptr[0] must be 0, rowptr
 *                      non-decreasing, 0 <= col < n.
 *   opt              : options (NULL = defaults)
 *   out              : receives the plan; NULL on failure
 * Errors: VP_EINVAL (n < 1, m < 1, non-finite coordinates or weights, bad
 * CSR, options out of range, a node or target outside a given root square,
 * out == NULL), VP_ENOMEM, VP_EDEVICE,
 * VP_EINTERNAL.  The tree is built on the device with this library's kernels.
 */
vp_status vp_plan(const double *x, const double *y, const double *w, int64_t n,
                  const double *tx, const double *ty, int64_t m,
                  const int64_t *rowptr, const int32_t *col, const double *val,
                  const vp_options *opt, vp_plan_t *out);

/*
 * Oversampled boxes (Section 4.2, eq. fk_basis and eq. Tnm: the density on a
 * box is its tensor-product Chebyshev interpolant of order p, given by its
 * values at the p x p roots of T_p, and the smooth rule sits at the q x q
 * roots of T_q, q >= p, the upsampling of Section 3.2 (the map O_{p,q} next
 * to eq. vals_to_coeffs); Section 4, eq. nsrcs, counts those q^2 sources per
 * box).  The caller gives the sources (the q x q nodes of every box, with
 * their smooth-rule weights), the targets, and which density values and
 * source nodes belong to each box; the library builds O (q^2 x p^2, the
 * tensor product of the 1D Chebyshev interpolation matrix) itself.  Within a
 * box, density value (ix, iy) sits at in_start[b] + iy*p + ix at the node
 * (c + h/2 xi_ix, c + h/2 xi_iy) and source (jx, jy) at out_start[b] +
 * jy*q + jx at (c + h/2 eta_jx, c + h/2 eta_jy), with xi / eta the roots of
 * T_p / T_q in ascending order, xi_i = -cos((2i+1) pi / 2p).
 */
typedef struct {
    int32_t p;                 /* density nodes per box side (1..32) */
    int32_t q;                 /* source nodes per box side (p..32) */
    int64_t nbox;              /* boxes; nbox * q * q must equal n */
    int64_t n_in;              /* density values per density (the length of f's rows) */
    const int64_t *in_start;   /* host [nbox]: first density value of box b (p*p values,
                                  disjoint between boxes, within [0, n_in)) */
    const int64_t *out_start;  /* host [nbox]: first source node of box b (q*q nodes,
                                  disjoint, together covering [0, n)) */
} vp_oversampling;

/*
 * vp_plan_oversampled -- as vp_plan, for the oversampled smooth rule:
 *   u[b][i] = sum_j G(r_j, t_i) w_j (O f[b])_j + sum_k C[i,k] f[b][k],
 * f [nbatch][n_in] the density values, O applied per box, C's columns index
 * the density values (0 <= col < n_in).  Targets must be given (tx, ty).
 * vp_eval / vp_eval_noalloc take f [nbatch][n_in]; vp_eval_adjoint returns
 * df [nbatch][n_in] = O^T (w * V^T g) + C^T g; vp_eval_grad_targets takes f
 * [nbatch][n_in].  Errors: as vp_plan, and VP_EINVAL for a layout outside the
 * rules above (os == NULL, p or q out of range, ranges out of bounds or
 * overlapping, sources not covered, no targets).
 */
vp_status vp_plan_oversampled(const double *x, const double *y, const double *w, int64_t n,
                              const double *tx, const double *ty, int64_t m,
                              const int64_t *rowptr, const int32_t *col, const double *val,
                              const vp_oversampling *os, const vp_options *opt, vp_plan_t *out);

/*
 * vp_eval -- u[b][i] = sum_j G(r_j, t_i) w_j f[b][j] + sum_k C[i,k] f[b][k].
 *   f [nbatch][n] device, u [nbatch][m] device; f and u must not overlap.
 */
vp_status vp_eval(vp_plan_t plan, const double *f, double *u);

/*
 * vp_eval_adjoint -- the exact transpose of vp_eval (used for dL/df):
 *   df[b][j] = w_j sum_i G(r_j, t_i) g[b][i] + sum_i C[i,j] g[b][i].
 *   g [nbatch][m] device, df [nbatch][n] device; no overlap.
 */
vp_status vp_eval_adjoint(vp_plan_t plan, const double *g, double *df);

/*
 * vp_eval_grad_targets -- gradient of the smooth sum with respect to the
 * target positions (the correction matrix is a fixed input and has none):
 *   grad[b][0][i] = d/dtx_i, grad[b][1][i] = d/dty_i of
 *   sum_j G(r_j, t_i) w_j f[b][j].
 *   f [nbatch][n] device, grad [nbatch][2][m] device; no overlap.
 */
vp_status vp_eval_grad_targets(vp_plan_t plan, const double *f, double *grad);

/*
 * vp_eval_noalloc -- vp_eval for callers that cannot allocate device memory
 * at evaluation time, nor have it allocated for them (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, result and stream semantics as vp_eval, with the same kernels;
 * the evaluation workspace (charges, multipole and local expansions, the
 * near- and far-field sums) lives in a static device array of the library
 * instead of the plan's own workspace, so the call allocates and frees
 * nothing (and calls no allocating library routine).
 *   Limit: the workspace must fit in VP_NOALLOC_MAX_BYTES (vp_get_info
 *   reports noalloc_bytes); a larger plan returns VP_EINVAL and does nothing.
 *   Every plan on a device shares that device's one array, which keeps the
 *   contents of the last call (each call clears what it needs zeroed): calls
 *   that overlap on one device (two streams, two host threads, or a call
 *   while an earlier one is still running on another stream) race and give
 *   wrong results.  Calls on one stream in sequence are safe.
 */
#define VP_NOALLOC_MAX_BYTES (64u << 20)
vp_status vp_eval_noalloc(vp_plan_t plan, const double *f, double *u);

/* Change the stream later evaluations run on (hipStream_t; NULL = null stream). */
vp_status vp_set_stream(vp_plan_t plan, void *stream);

/* Release the plan's device memory (synchronises its stream).  NULL is a no-op. */
vp_status vp_destroy(vp_plan_t plan);

/* Message of the last error on this plan, or of the calling thread's last
 * vp_plan failure when plan is NULL.  Never NULL; valid until the next call. */
const char *vp_last_error(vp_plan_t plan);

/* Sizes of a built plan, for callers and tests. */
typedef struct {
    int64_t n, m, nnz;
    int32_t nbatch, order, precision, m2l_mode, p2p_mode_used, max_leaf;
    int32_t nbox, nleaf, nlevels, self_targets;
    int64_t list_len[4];       /* total entries of the U, V, W, X lists */
    int64_t table_leaves;      /* leaves served by near-field tables */
    int64_t near_pairs;        /* (target, source) pairs the pairwise near-field kernel evaluates
                                  per density in the forward sum */
    int64_t workspace_bytes;   /* device memory held by the plan */
    int64_t m2l_translations;  /* M2L translations per density, V lists plus the
                                  virtual children of X-list sources */
    int64_t m2l_tile_ops;      /* (16-column tile, offset) products the M2L launches issue */
    int64_t table_tile_ops;    /* (16-column tile, slot) products of the near tables */
    int64_t m2l_coarse_translations;  /* of m2l_translations, those into boxes below split_level */
    int64_t m2l_coarse_tile_ops;      /* of m2l_tile_ops, those of the launch below split_level */
    int32_t split_level;       /* expansion passes of the levels below it run on a third stream
                                  beside the M2L of the levels from it on (2: none below) */
    int32_t corr_cells;        /* cells of C applied cell by cell (consecutive rows sharing one
                                  column run); 0: the row kernel applies C */
    int32_t corr_shared_cells; /* of corr_cells, those whose value block is bit for bit that of an
                                  earlier cell and which read that cell's copy (the box corrections
                                  of one box size are one table, Section 4) */
    int64_t corr_values_read;  /* distinct values of C one forward apply reads: nnz less the
                                  values of the shared cells */
    int32_t corr_groups;       /* one density: groups of up to 16 64-column cells reading one
                                  block, applied together on the matrix cores (0: none) */
    int32_t corr_one_block;    /* 1: every cell is a 64 x 64 block reading one shared block, and C is
                                  applied as that one fixed operator on the matrix cores */
    double root[3];
    int64_t table_pairs;       /* (target, source) pairs per density served by the near-field
                                  tables (near_pairs holds the pairwise kernel's) */
    int64_t noalloc_bytes;     /* static workspace vp_eval_noalloc needs for this plan */
    int64_t n_in;              /* density values per density (n unless oversampled) */
    int32_t os_p, os_q;        /* oversampled plan: nodes per box side (0, 0: none) */
    int32_t kernel;            /* VP_KERNEL_* */
    int32_t table_pattern;     /* points per pattern leaf of the near-field tables (0: no tables) */
    double lambda;
    int32_t tuned;             /* 0: defaults; 1: tuned by timing in this call; 2: from the cache */
    int32_t m2l_waves;         /* waves per 16-column tile of the M2L kernels */
    int32_t table_waves;       /* waves per tile of the near-table kernel */
    int32_t one_stream;        /* 1: every kernel of an evaluation on the plan's stream */
    double tune_ms;            /* plan time spent timing candidates */
    int32_t l2p_from_parents;  /* 1: forward evaluations evaluate the deepest level's pattern leaves
                                  from their parents' local expansions (L2L into that level folded
                                  into the L2P matrices; uniform grids, densities a multiple of 16) */
    int32_t corr_folded;       /* 1: forward evaluations apply the own-cell corrections inside the
                                  near-field tables (one shared block on congruent leaves: the self
                                  slot's matrix becomes the leaf's own-cell quadrature, Section 4);
                                  the correction pass is skipped */
} vp_plan_info_t;

vp_status vp_get_info(vp_plan_t plan, vp_plan_info_t *info);

/*
 * Introspection for tests: copy one plan array to host memory (synchronous).
 *   which: VP_ARR_* below; out must hold the advertised count of elements of
 *   the stated type (query with out == NULL: *count receives the length).
 */
enum {
    VP_ARR_SRC_PERM = 0,   /* int32 [n]      sorted position -> node index    */
    VP_ARR_TGT_PERM = 1,   /* int32 [m]      sorted position -> target index  */
    VP_ARR_BOX = 2,        /* int32 [nbox][10]: level, ix, iy, parent,
                              child_begin (-1 leaf), nchild, src_begin,
                              src_end, tgt_begin, tgt_end                     */
    VP_ARR_LEVEL_BEGIN = 3,/* int32 [nlevels+1]                               */
    VP_ARR_U_PTR = 4, VP_ARR_U_IDX = 5,  /* int32 CSR over boxes (sorted)     */
    VP_ARR_V_PTR = 6, VP_ARR_V_IDX = 7,
    VP_ARR_W_PTR = 8, VP_ARR_W_IDX = 9,
    VP_ARR_X_PTR = 10, VP_ARR_X_IDX = 11,
    VP_ARR_MULTIPOLE = 12, /* float64 [nbox][nbatch][2][p+1] (re, im) after the
                              last vp_eval (float32 forms are widened)        */
    VP_ARR_LOCAL = 13,     /* same layout: local expansions after the last
                              vp_eval's downward pass                         */
    VP_ARR_SRC_KEYS = 14,  /* int64 [n] sorted Morton keys                    */
    VP_ARR_TGT_KEYS = 15   /* int64 [m]                                       */
};
vp_status vp_get_array(vp_plan_t plan, int32_t which, void *out, int64_t *count);

/*
 * Per-stage device timing of evaluations (profiling aid).  When enabled, each
 * stage of vp_eval / vp_eval_adjoint / vp_eval_grad_targets is bracketed by
 * HIP events recorded on the plan's stream (no host synchronisation inside
 * the evaluation).  vp_set_timing(plan, 1) creates the events and clears the
 * accumulators, (plan, 0) releases them.  vp_get_timing synchronises the
 * stream and returns the summed milliseconds per stage (ms[VP_NSTAGES]) and
 * the number of timed evaluations.
 */
enum {
    VP_STAGE_CHARGE = 0, VP_STAGE_P2M = 1, VP_STAGE_M2M = 2, VP_STAGE_M2L = 3, VP_STAGE_P2L = 4,
    VP_STAGE_L2L = 5, VP_STAGE_P2P = 6, VP_STAGE_FAR = 7, VP_STAGE_FINISH = 8,
    VP_STAGE_TABLES = 9, /* near-field tables of congruent leaves (P2P holds the pairwise kernel) */
    VP_STAGE_CORR = 10,  /* sparse correction apply C f (FINISH: adding the un-permuted FMM sums) */
    VP_STAGE_COARSE = 11,/* M2M, M2L and L2L of the levels below split_level (third stream);
                            M2M, M2L and L2L hold the levels from split_level on */
    VP_STAGE_P2M_PAT = 12,/* P2M by fixed matrices (pattern leaves and their quadrants);
                             P2M holds the VALU P2M of the other leaves (third stream) */
    VP_STAGE_M2P = 13,   /* W-list multipoles at the targets (second stream, between the
                            tables and the pairwise kernel); FAR holds the local expansions
                            at the targets (with gradients: both) */
    VP_NSTAGES = 14
};
vp_status vp_set_timing(vp_plan_t plan, int32_t enable);
vp_status vp_get_timing(vp_plan_t plan, double *ms, int64_t *nevals);

/*
 * vp_correction_blocks -- own-cell singular corrections generated on the
 * device (Section 4.1, eqs. maptri_singular_quad and singcorr_inner_prod;
 * Section 4.2, eqs. mapbox_singular_quad and Vkhat_box).
 *
 * Cells are affine images r = o_k + A_k zeta of one reference cell carrying
 * one node pattern zeta_j: VP_CELL_BOX ([-1,1]^2, interpolation by
 * polynomials of degree < p in each variable, N = p^2 nodes) or
 * VP_CELL_TRIANGLE (the simplex xi, eta >= 0, xi + eta <= 1, total degree
 * < p, N = p(p+1)/2 nodes).  For cell k, with nodes r_j = o_k + A_k zeta_j and
 * smooth weights w_j = |det A_k| wref_j, entry (i, j) of block k is
 *
 *     C_ij = int_cell G(r, r_i) l_j(r) dA(r)  -  [j != i] G(r_j, r_i) w_j,
 *
 * l_j the Lagrange basis of the interpolation space on the pattern: the
 * correction that turns the smooth rule's sum over the cell into the exact
 * integral of G against the interpolant of f (the paper writes the same map
 * through the interpolant's coefficients, V a = f, and the singular integrals
 * of the basis).  Row i of a block is the own-cell row of target r_i in the
 * correction matrix C of vp_plan.
 *
 * The singular integrals: the reference cell is split at the target into
 * triangles with the target as apex; on each, log|A (zeta - zeta_i)| = log u +
 * log|A d(v)| for zeta = zeta_i + u d(v), the u integral is exact (16
 * Gauss-Legendre points with weights for u and for u log u; polynomials of
 * degree < 16 along a ray) and the v integral is composite 12-point
 * Gauss-Legendre graded toward the point of the edge nearest the target in
 * physical space.  Agreement with direct high-precision integration is near
 * 1e-14 of the largest entry of a block.
 *
 * shape, p      VP_CELL_BOX with 1 <= p <= 8, or VP_CELL_TRIANGLE with
 *               1 <= p <= 10 (VP_EUNSUPPORTED above).
 * ref_x, ref_y  HOST [N]: the pattern in reference coordinates, every node at
 *               least 1e-9 inside the reference cell, unisolvent for the space.
 * wref          HOST [N]: smooth weights in reference coordinates.
 * ncell         number of cells, >= 0 (ncell * N below 2^31).
 * maps          DEVICE [ncell][6]: o_x, o_y, A_00, A_01, A_10, A_11 per cell
 *               (r = o + A zeta, A row-major), det A != 0; read, not modified.
 * out           DEVICE [ncell][N][N]: block k, row i, column j; overwritten.
 * stream        hipStream_t for the copies and the kernel (NULL: the null
 *               stream).  The call builds the rule tables on the host, copies
 *               them and the maps' check to and from the device, runs the
 *               kernel and synchronises the stream before returning (it
 *               allocates and frees one small device table: a set-up call).
 * Errors: VP_EINVAL (message from vp_last_error(NULL)) for a NULL pointer, a
 * node outside the cell, a pattern that is not unisolvent, a non-finite or
 * singular map; VP_EUNSUPPORTED for an order outside the ranges above;
 * VP_EDEVICE for a HIP error.  Nothing is written on VP_EINVAL.
 */
enum { VP_CELL_BOX = 0, VP_CELL_TRIANGLE = 1 };
vp_status vp_correction_blocks(int32_t shape, int32_t p, const double *ref_x, const double *ref_y,
                               const double *wref, int64_t ncell, const double *maps, double *out,
                               void *stream);

#ifdef __cplusplus
}
#endif

#endif /* VP_H */

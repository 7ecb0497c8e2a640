// Internal declarations of libvp: the plan object, error plumbing, device
// helpers shared by the tree, FMM and correction kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/vp.h"

namespace vp {

// ----------------------------------------------------------------------------
// Errors.  Internal code throws; the C ABI catches and maps to vp_status.
// ----------------------------------------------------------------------------
struct Error : std::runtime_error {
    vp_status status;
    Error(vp_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] void throw_hip(hipError_t e, const char *expr, const char *file, int line);

#define VP_HIP(expr)                                                   \
    do {                                                               \
        hipError_t _vp_e = (expr);                                     \
        if (_vp_e != hipSuccess) ::vp::throw_hip(_vp_e, #expr, __FILE__, __LINE__); \
    } while (0)

#define VP_LAUNCH_CHECK() VP_HIP(hipGetLastError())

// ----------------------------------------------------------------------------
// Constants
// ----------------------------------------------------------------------------
constexpr int LBITS = 30;              // quantisation bits per coordinate
constexpr int QI_ZERO_PTS = 128;         // zero points after the density-fastest charges
constexpr int NOFF = 40;               // M2L offsets: [-3,3]^2 minus [-1,1]^2
constexpr int MAX_BATCH = 64;
constexpr double INV_2PI = 0.15915494309189533576888376337251436;
constexpr double INV_4PI = 0.07957747154594766788444188168625718;
constexpr double LN2_4PI = 0.05515890003816289834911410802949942;  // log(2) / (4 pi)

// offset code of (dx, dy) in [-3,3]^2 with max(|dx|,|dy|) >= 2, else -1
__host__ __device__ inline int offset_code(int dx, int dy) {
    if (dx < -3 || dx > 3 || dy < -3 || dy > 3) return -1;
    if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) return -1;
    int c = (dy + 3) * 7 + (dx + 3);  // 0..48
    // remove the 9 inner codes (dy in -1..1, dx in -1..1) from the numbering
    int inner_before = 0;
    if (dy > 1) inner_before = 9;
    else if (dy >= -1) inner_before = (dy + 1) * 3 + (dx > 1 ? 3 : 0);
    return c - inner_before;
}

// ----------------------------------------------------------------------------
// Device memory owned by a plan
// ----------------------------------------------------------------------------
struct DeviceArena {
    std::vector<void *> ptrs;
    size_t bytes = 0;
    template <class T>
    T *alloc(size_t count) {
        if (count == 0) count = 1;
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(VP_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
        }
        ptrs.push_back(p);
        bytes += count * sizeof(T);
        return static_cast<T *>(p);
    }
    void release(void *p) {
        for (auto &q : ptrs)
            if (q == p) {
                (void)hipFree(q);
                q = nullptr;
            }
    }
    void free_all() {
        for (void *p : ptrs)
            if (p) (void)hipFree(p);
        ptrs.clear();
        bytes = 0;
    }
};

// Temporary device buffers freed at scope exit (plan time only).
struct TempArena {
    std::vector<void *> ptrs;
    template <class T>
    T *alloc(size_t count) {
        if (count == 0) count = 1;
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(VP_ENOMEM, "hipMalloc (temporary) failed");
        }
        ptrs.push_back(p);
        return static_cast<T *>(p);
    }
    ~TempArena() {
        for (void *p : ptrs) (void)hipFree(p);
    }
};

// ----------------------------------------------------------------------------
// Tree and lists as held on the device
// ----------------------------------------------------------------------------
struct Tree {
    int nbox = 0, nlevels = 0, nleaf = 0;
    std::vector<int32_t> level_begin;  // host copy, nlevels+1
    std::vector<double> side;          // host, per level
    int32_t *d_level_begin = nullptr;
    int32_t *level = nullptr, *ix = nullptr, *iy = nullptr, *parent = nullptr;
    int32_t *child = nullptr, *nchild = nullptr;
    int32_t *sb = nullptr, *se = nullptr, *tb = nullptr, *te = nullptr;
    uint64_t *key = nullptr;           // Morton key of (ix, iy) on its level
    double *cx = nullptr, *cy = nullptr;
    double *d_side = nullptr;          // per level
    double *d_logside = nullptr;       // per level
    int32_t *leaves = nullptr;         // leaf box indices
    // lists, CSR over all boxes
    int32_t *lptr[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t *lidx[4] = {nullptr, nullptr, nullptr, nullptr};
    int64_t llen[4] = {0, 0, 0, 0};
    int32_t *v_off = nullptr;          // offset code of each V entry
    int32_t *v_slot = nullptr;         // [nbox][NOFF] source box or -1
};

// Translation operators in real PD x PD form (see vp_ops.cpp).
struct Operators {
    int P = 0, PD = 0;
    // A-fragment order for the MFMA kernels: [op][rb][s][lane]
    double *m2l_f64 = nullptr;  // NOFF ops
    float *m2l_f32 = nullptr;
    float *m2l_f32_lo = nullptr;
    // M2M / L2L in diagonally scaled form (index 0 = M2M, 1 = L2L): a real
    // P x P matrix stored transposed, QT[k][l] with row stride PR (power of
    // two >= P), and per child class complex scalings tin[c][k], tout[c][l]
    // ([4][P][2])
    int PR = 0;
    double *sh_qt64[2] = {nullptr, nullptr}, *sh_tin64[2] = {nullptr, nullptr}, *sh_tout64[2] = {nullptr, nullptr};
    float *sh_qt32[2] = {nullptr, nullptr}, *sh_tin32[2] = {nullptr, nullptr}, *sh_tout32[2] = {nullptr, nullptr};
    double *log_table = nullptr;  // [LOG_TABLE][2]: fl(1/c_i), -log2(fl(1/c_i)) (pairwise logarithm)
    double *inv_k = nullptr;  // 1/k, k = 0..P-1 (0 for k = 0)
    float *inv_k_f32 = nullptr;
    // M2L in diagonally scaled form: one real matrix Q (A-fragment order,
    // PQ = roundup(P, 16) rows and columns), per-offset complex scalings
    // tin[o][k] = (-t)^-k and tout[o][l] = t^-l ([NOFF][PQ][2]), log(-t)
    int PQ = 0;
    double *m2l_q64 = nullptr, *m2l_tin64 = nullptr, *m2l_logt = nullptr;  // scaled M2L (Q rows signed)
    float *m2l_q32 = nullptr, *m2l_tin32 = nullptr;
};

// near-field table slots per target level: 9 same level, 16 coarser, 16 finer
constexpr int NTOPS = 41;
// logarithm table of the pairwise near field: LOG_BITS top fraction bits of
// the mantissa select one of LOG_TABLE entries
constexpr int LOG_BITS = 7;
constexpr int LOG_TABLE = 1 << LOG_BITS;

// Pairwise near-field sources of a list of target leaves, gathered once at
// plan time (static geometry): for leaf k of the list, entries
// [ptr[k], ptr[k+1]) hold the sorted indices and coordinates of every source
// point in its U list, in list order, so the kernel stages them with
// contiguous loads.
struct P2PGather {
    int64_t *ptr = nullptr;
    int32_t *idx = nullptr;
    double *x = nullptr, *y = nullptr;
    int64_t len = 0;
};

// One VALU P2M job: sources [s0, s1) (sorted order) about (cx, cy) at scale
// 1 / inv_s into expansion column col (a leaf, or a virtual child nbox + 4 v + q).
struct P2MJob {
    double cx, cy, inv_s;
    int32_t s0, s1, col, pad;
};

// One M2L launch over the boxes of a range of levels: (box, density)
// columns in 16-column tiles, with the offsets present in each tile and each
// column's source box per offset.
struct M2LSched {
    int32_t *cols = nullptr;    // boxes, grouped by child class, then by their set of offsets
    int nboxes = 0;
    int32_t *tptr = nullptr;    // offsets of tile t: tops[tptr[t] .. tptr[t+1])
    int32_t *tops = nullptr;
    int32_t *tsrc = nullptr;    // [tile offset][16] source box per column, or -1
    int32_t *torder = nullptr;  // tiles by decreasing offset count
    int32_t *torder4 = nullptr; // the same, dealt to the XCDs in groups of four tiles (one wave per tile)
    int64_t translations = 0, tile_ops = 0;
};

// Congruent-leaf path (uniform box grids): near-field tables, P2M/L2P
// operators of the node pattern, and the leftover pairwise lists.
struct NearTables {
    bool active = false;
    int npat = 0;                     // points per pattern leaf
    int nleaf_tab = 0;                // target leaves with at least one table slot
    std::vector<int> tab_levels;      // levels holding table columns
    std::vector<int> tab_cols_begin;  // per entry of tab_levels, offsets into tab_cols
    int32_t *tab_cols = nullptr;      // table target leaves, grouped by level
    int32_t *tab_slot = nullptr;      // [nbox][41 * table levels] table source per slot or -1
    int32_t *tile_ptr = nullptr;      // slots present per 16-column tile of table columns
    int32_t *tile_ops = nullptr;
    int32_t *tile_order = nullptr;    // tiles by decreasing operator count
    int32_t *tile2_ptr = nullptr;     // the same over 32-column groups (one wave over two tiles)
    int32_t *tile2_ops = nullptr;
    int32_t *tile2_order = nullptr;
    int64_t table_tile_ops = 0;
    double *K = nullptr;              // [tab level][41] near matrices, A-fragment order
    // forward evaluations with the own-cell corrections folded into the self
    // slot (K_self + C W^-1 on the charges W f): K with that slot replaced
    double *Kf = nullptr;
    bool corr_folded = false;
    int32_t *pair_uptr = nullptr;     // U lists minus the table-served entries
    int32_t *pair_uidx = nullptr;
    int64_t rest_len = 0;
    int32_t *rest_leaves = nullptr;   // leaves with a non-empty leftover list
    int n_rest_leaves = 0;
    P2PGather g_rest;                 // sources of the leftover lists
    int32_t *ident_slot = nullptr;    // [nbox] slot table b -> b (one-operator launches)
    // P2M by fixed matrices: pattern leaves (operator 0), then the virtual
    // children of pattern X-list sources grouped by quadrant (operator 1 + q)
    int32_t *p2m_cols = nullptr;
    int n_p2m_cols = 0;
    int n_p2m_leaf_cols = 0;          // of p2m_cols, the leading pattern leaves (operator 0)
    int32_t *p2m_slot = nullptr;      // [nbox + 4 n_vleaf][5] source leaf in the column's operator slot, or -1
    P2MJob *p2m_jobs_rest = nullptr;  // VALU P2M jobs of the rest (source role)
    int n_p2m_jobs_rest = 0;
    int32_t *l2p_pat = nullptr;       // pattern target leaves (level >= 2)
    int n_l2p_pat = 0;
    int32_t *far_leaves = nullptr;    // leaves needing the series far-field kernel
    int n_far_leaves = 0;
    int32_t *l2p_rest = nullptr;      // leaves (level >= 2) whose local expansion is evaluated by the series
    int n_l2p_rest = 0;
    int32_t *local_done = nullptr;    // [nbox] 1: local expansion evaluated by the L2P operator
    // leaves whose near / far sums are zeroed before their first (adding)
    // writer; the tables and the pattern L2P store the others
    int32_t *zero_near = nullptr, *zero_far = nullptr;
    int n_zero_near = 0, n_zero_far = 0;
    int32_t *far_add = nullptr;       // [nbox] 1: the pattern L2P adds (W lists wrote first); null: none
    bool fused_finish = false;        // forward: the pattern L2P writes the output (see vp_near.hip)
    // forward with the fused finish: the pattern leaves fill the deepest level
    // par_level, whose L2P starts from the parents' local expansions (the L2L
    // into that level folded into par_km, one matrix per child class)
    bool par_l2p = false;
    int par_level = 0;
    double *l2p_km = nullptr;         // L2P (npat x PD), k-major fragments
    double *par_km = nullptr;         // [4] B_q = L2P x L2L_q, k-major fragments
    int32_t *l2p_rec = nullptr;       // [tile][4] {box, parent * 4 + class, first density, 0}, by class
    int l2p_qbeg[5] = {0, 0, 0, 0, 0};  // class q's tiles: [l2p_qbeg[q], l2p_qbeg[q + 1])
    std::vector<double> pat_rx, pat_ry;  // the node pattern, box-relative in units of the side
    // [5][PD x npat] A-fragment order: the leaf P2M, then the four quadrant
    // P2M matrices (about the quadrant centre at the children's scale, zero
    // outside the quadrant's points)
    double *p2m_op = nullptr, *l2p_op = nullptr;      // float64 forms
    float *p2m_op_f32 = nullptr, *l2p_op_f32 = nullptr;  // FP32-bulk forms
};

// Modified Helmholtz kernel (vp_yukawa.hip): fixed matrices per level on a
// uniform grid of congruent leaves
struct YukawaPlan {
    bool active = false;
    double lambda = 0.0, cG = 0.0;   // G = cG K_0(lambda r), cG = lambda^2 / (2 pi)
    int leaf_level = -1;
    double *p2m = nullptr, *l2p = nullptr;            // pattern operators, A-fragment order
    double *m2m = nullptr, *l2l = nullptr;            // [level][child quadrant] PD x PD
    double *m2l = nullptr;                            // [level][offset code] PD x PD
    int32_t *cslot = nullptr;                         // [nbox][4] child in each quadrant (M2M)
    int32_t *pslot = nullptr;                         // [nbox][4] parent in the box's quadrant slot (L2L)
    std::vector<std::vector<int32_t>> parents, children;  // per level (host)
    std::vector<int32_t *> d_parents, d_children;
    int32_t *m2l_cols = nullptr, *m2l_slot = nullptr;     // boxes of level >= 2; [nbox][NOFF x nlevels]
    int32_t *m2l_tptr = nullptr, *m2l_tops = nullptr, *m2l_torder = nullptr;
    int n_m2l_cols = 0;
    int64_t m2l_translations = 0, m2l_tile_ops = 0;
};

}  // namespace vp

// ----------------------------------------------------------------------------
// The plan
// ----------------------------------------------------------------------------
struct vp_plan_s {
    vp_options opt{};
    int p = 30, P = 31, PD = 64;
    int64_t n = 0, m = 0, nnz = 0;
    int64_t nd = 0;          // density values per density: n, or n_in of an oversampled plan
    // oversampled boxes (vp_plan_oversampled): per box, p x p density values
    // -> q x q source nodes by the tensor-product Chebyshev map O (q^2 x p^2)
    int os_p = 0, os_q = 0;  // 0: no oversampling (the density is given at the sources)
    int64_t os_nbox = 0;
    int64_t *os_in = nullptr, *os_out = nullptr;  // [os_nbox] first density value / first source node
    double *os_O = nullptr;   // [q^2][p^2] row-major (adjoint: threads over columns)
    double *os_OT = nullptr;  // [p^2][q^2] (forward: threads over rows)
    int nbatch = 1;
    bool self = false;
    bool fp32 = false;
    int m2l_mode = VP_M2L_FP64_MFMA;
    int m2l_nw = 1;           // waves per 16-column tile of the M2L kernels (4, 2, or 1: one wave per tile)
    int table_nw = 1;         // waves per tile of the near-table launch (1: one wave over two tiles)
    int tuned = 0;            // 0: defaults; 1: chosen by timing at plan time; 2: from the tuning cache
    double tune_ms = 0.0;     // plan time spent tuning
    bool one_stream = false;  // no second stream: every kernel on the plan's stream
    hipStream_t stream = nullptr;
    // the near field runs on its own stream, forked after the charges and
    // joined before the far-field evaluation (both default priority)
    hipStream_t aux = nullptr;
    // third stream: P2L, then the expansion passes of the levels below
    // split_level (few boxes, latency bound) beside the M2L of the levels above
    hipStream_t aux2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_p2m = nullptr, ev_p2l = nullptr, ev_upper = nullptr, ev_coarse = nullptr, ev_m2p = nullptr;
    int device = 0;
    std::string err;
    bool poisoned = false;

    vp::DeviceArena mem;
    // points in sorted (Morton) order
    double *sx = nullptr, *sy = nullptr, *sw = nullptr;
    int32_t *sperm = nullptr, *sinv = nullptr;
    uint64_t *skeys = nullptr;
    double *tx = nullptr, *ty = nullptr;
    int32_t *tperm = nullptr, *tinv = nullptr;
    uint64_t *tkeys = nullptr;
    double *w_user = nullptr;  // weights in user order (adjoint)
    // correction matrix (user order) and its transpose
    int64_t *rowptr = nullptr;
    int32_t *col = nullptr;
    double *val = nullptr;
    int64_t *rowptrT = nullptr;
    int32_t *colT = nullptr;
    double *valT = nullptr;
    int32_t *run_start = nullptr;   // per row: first column of a contiguous run, or -1
    bool all_runs = false, all_runsT = false;  // every row (of C, of C^T) is a run
    int32_t *run_startT = nullptr;
    // cells (consecutive rows sharing one column run of <= 64): [ncell + 1]
    // first rows, [ncell] first columns; ncell = 0: the row kernel applies C
    int32_t *cell_row = nullptr, *cell_col = nullptr, *cell_rowT = nullptr, *cell_colT = nullptr;
    int ncell = 0, ncellT = 0;
    // offset of the values each cell reads: its own, or those of the first
    // cell with an identical block (found at plan time, compared exactly)
    int64_t *cell_vb = nullptr, *cell_vbT = nullptr;
    int ncell_shared = 0;           // cells reading another cell's identical block
    // one density: groups of up to 16 64-column cells reading one block
    // (cell ids, -1 padded; value offset and rows per group), and the offsets
    // the cell kernel uses then (-1: the cell is applied by its group)
    int32_t *grp_cell = nullptr, *grp_cellT = nullptr, *grp_rows = nullptr, *grp_rowsT = nullptr;
    int64_t *grp_vb = nullptr, *grp_vbT = nullptr, *cell_vbg = nullptr, *cell_vbgT = nullptr;
    int ngrp = 0, ngrpT = 0;
    int64_t corr_values_read = 0;   // values the forward apply reads from memory
    // every cell one shared 64 x 64 block: that block in A-fragment order (else null)
    double *corr_op = nullptr, *corr_opT = nullptr;
    // the same forward block row-major on the host, with the cells' first
    // rows ([ncell + 1]) and first columns (for folding C into the near tables)
    std::vector<double> corr_block;
    std::vector<int32_t> corr_cell_row, corr_cell_col;
    int32_t *cell_iota = nullptr;   // 0, 1, 2, ... (the cells as the fixed-operator kernel's columns)
    int n_cell_iota = 0;

    vp::Tree tree;
    vp::Operators ops;
    vp::NearTables near;
    vp::YukawaPlan yk;
    int64_t near_pairs = 0;
    int64_t table_pairs = 0;

    // evaluation workspace
    double *q = nullptr;     // [nbatch][max(n,m)] charges, sorted order
    double *acc = nullptr;   // [nbatch][max(n,m)] potentials, sorted order (near field; gradients x 2)
    double *acc_far = nullptr;  // [nbatch][max(n,m)] far-field potentials, sorted order
    double *qi = nullptr;    // [max(n,m) + QI_ZERO_PTS][nbatch] the charges again, density fastest (near
                             // tables, nbatch > 1); the last QI_ZERO_PTS points stay zero (an absent source)
    int64_t qi_zero = 0;     // point index of that zero block (max(n, m))
    // forward evaluations with the near tables whose only other reader of the
    // charges is the pattern P2M of the leaves (no VALU P2M, quadrant P2M, P2L
    // or leftover pairwise work): the pattern P2M then reads qi and q is not
    // written (q_valid false)
    bool q_pattern_only = false;
    bool q_valid = true;
    bool qi_valid = false;   // qi holds this evaluation's charges
    bool p2m_in_charges = false;  // this evaluation's charge pass also formed the leaf multipoles
    void *Mexp = nullptr;    // [mexp_boxes()][nbatch][PD] (double or float)
    void *Lexp = nullptr;
    void *zero_col = nullptr;  // max(PD, 128 nbatch) zero doubles (an absent source column, either element
                               // type and either charge layout)
    void *scratch_dev = nullptr;  // this device's static workspace (vp_eval_noalloc), resolved at plan time
    vp::P2PGather g_fwd, g_adj;   // full U-list sources (nodes / targets as sources) without tables
    // M2L launches: [0] levels >= split_level, [1] levels 2 .. split_level-1
    vp::M2LSched m2l[2];
    int split_level = 2;
    int64_t m2l_translations = 0, m2l_tile_ops = 0;  // both launches
    int32_t *x_init = nullptr;  // [nbox] 1: P2L writes the local expansion before M2L adds to it
    int32_t *m2m_cslot = nullptr;    // [m2m_parents][4] child in each quadrant or -1
    int32_t *lvl_pcls = nullptr;     // [lvl_boxes] parent * 4 + class
    int32_t *lvl_boxes = nullptr;  // boxes of each level, grouped by class inside a level (L2L)
    std::vector<int> lvl_box_begin;  // per level offsets into lvl_boxes
    int32_t *m2m_parents = nullptr;  // non-leaf boxes per level
    std::vector<int> m2m_begin;
    // VALU P2M jobs without tables: leaves of level >= 2, then the virtual
    // children of X-list sources, for the nodes and for the targets as sources
    vp::P2MJob *p2m_jobs = nullptr, *p2m_jobs_t = nullptr;
    int n_p2m_jobs = 0;
    int32_t *x_boxes = nullptr;      // boxes whose X list keeps entries for the P2L kernel
    int n_x_boxes = 0;
    int32_t *xr_ptr = nullptr;       // those X entries (two or more levels apart), CSR over boxes
    int32_t *xr_idx = nullptr;
    // X-list source leaves one level above their targets: four virtual
    // children each (expansion columns nbox + 4 v + quadrant), with the
    // quadrant boundaries [5] of their sorted sources and targets
    int n_vleaf = 0;
    int32_t *vleaf = nullptr;
    // multipole blocks: the boxes, the virtual children, and one block that
    // stays zero (index zero_box(): the M2L's absent source)
    int64_t zero_box() const { return (int64_t)tree.nbox + 4 * (int64_t)n_vleaf; }
    int64_t mexp_boxes() const { return zero_box() + 1; }
    int32_t *vsplit_s = nullptr, *vsplit_t = nullptr;
    int32_t *w_leaves = nullptr;     // leaves with non-empty W list
    int n_w_leaves = 0;
    int32_t *err_flag = nullptr;     // device error flag (list traversal overflow)

    // optional per-stage timing (HIP events on the plan's stream)
    static constexpr int TRING = 32;
    bool timing = false;
    std::vector<hipEvent_t> tev;     // [TRING][VP_NSTAGES][2]
    std::vector<int> tslot_used;     // stages recorded in a ring slot (bit mask)
    int64_t tcount = 0;              // evaluations started with timing on
    int64_t tdone = 0;               // evaluations folded into tms
    double tms[VP_NSTAGES] = {0};
    int tcur = -1;
    void stage_begin(int st);
    void stage_end(int st);
    void timing_eval_begin();
    void timing_collect(int64_t upto);
};

void vp_to_frag(const double *R, int rows, int cols, int ld, double *F);
void vp_to_frag_kmajor(const double *R, int rows, int cols, int ld, double *F);

namespace vp {
// vp_tree.hip
void build_tree(vp_plan_s *P, const double *hx, const double *hy, const double *htx,
                const double *hty);
// vp_ops.cpp
void build_operators(vp_plan_s *P);
// vp_near.hip
void build_near_tables(vp_plan_s *P);  // vp_near.hip
// vp_yukawa.hip: operators and lists of the modified Helmholtz kernel
void build_yukawa(vp_plan_s *P);
// vp_fmm.hip
void build_schedules(vp_plan_s *P);
// plan-time autotuner (M2L form and waves per tile, near-table waves per
// tile, streams), each candidate timed on full evaluations; returns the best ms
float autotune(vp_plan_s *P);
// wall time of one forward evaluation (the smallest of reps after a warm-up)
float time_forward(vp_plan_s *P, const double *f, double *u, int reps);
// P2M job descriptors for job codes (leaf b >= 0, or ~(4 v + quadrant)) in
// the source role (nodes) or the target role (targets as sources)
std::vector<P2MJob> p2m_job_descs(vp_plan_s *P, const std::vector<int32_t> &codes, bool target_role);
// congruent-leaf operators exist for this pattern size and expansion size
bool pattern_op_supported(int npat, int PD);
// gather the U-list sources of `leaves` (host CSR uptr/uidx, source ranges sb/se; device coordinates sx/sy)
void build_p2p_gather(vp_plan_s *P, const std::vector<int32_t> &leaves, const std::vector<int32_t> &uptr,
                      const std::vector<int32_t> &uidx, const std::vector<int32_t> &sb, const std::vector<int32_t> &se,
                      const double *sx, const double *sy, P2PGather &g);
// own-cell singular correction blocks of affine cells (vp_correction_blocks)
void correction_blocks(int shape, int p, const double *ref_x, const double *ref_y, const double *wref,
                       int64_t ncell, const double *maps, double *out, hipStream_t stream);
// launch order of tiles with tile_ptr[t+1] - tile_ptr[t] operators: most operators
// first, dealt to the XCDs in runs of workgroups of `group` consecutive tiles
std::vector<int32_t> tile_order_by_work(const std::vector<int32_t> &tile_ptr, int group = 1);
// one evaluation after prepare_charges; with u: the correction C f (adjoint C^T f) runs
// beside the FMM and u = FMM sums (un-permuted; adjoint: times w) + correction
void run_fmm(vp_plan_s *P, bool adjoint, bool grad, const double *f = nullptr, double *u = nullptr);
// grad: the evaluation forms target gradients (its near field reads q)
void prepare_charges(vp_plan_s *P, const double *f, bool adjoint, bool grad = false);
void finish_grad(vp_plan_s *P, double *grad);
void detect_runs(vp_plan_s *P);
// vp_csr.hip
void build_csr_transpose(vp_plan_s *P);
// utilities (vp_tree.hip)
void exclusive_scan_i32(const int32_t *in, int32_t *out, int n, hipStream_t s);
void radix_sort_pairs_u64(uint64_t *keys, int32_t *vals, int n, int nbits, hipStream_t s);
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
void fill_f64(double *p, double v, int64_t n, hipStream_t s);
void fill_f32(float *p, float v, int64_t n, hipStream_t s);
}  // namespace vp

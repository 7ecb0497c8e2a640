// Gather-GEMM on matrix cores: the one kernel behind every dense, fixed-
// operator step of the evaluation.
//
//   out[:, col] (+)= sum_o A_o in[:, src(col, o)]
//
// A column is a (box, density) pair; src(col, o) is the box in slot o of the
// column's box (or none).  Uses:
//   M2L          40 outer offsets, A_o = M2L operator (+ the A_0 log s row):
//                the per-offset form, k_translate_split (the default M2L is
//                the diagonally scaled kernel of vp_m2l_scaled.hpp)
//   near tables  neighbour positions of congruent leaves, A_o = G matrix
//                (k_translate_split)
//   P2M          5 operators on congruent leaves (leaf and quadrants, k_translate)
//   L2P          1 operator on congruent leaves (k_pattern_op)
// k_translate stages the operator of the current slot once in LDS and shares
// it between the four waves of a workgroup, each wave owning 16 columns.
// Operators are stored in A-fragment order [o][rb][s][lane], element
// (row rb*16 + l%16, k = 4 s + l/16), so staging is a straight coalesced copy.
#pragma once

#include "vp_internal.hpp"

namespace vp {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Column addressing: element r of the column (box a, density b) is at
// base + off(a) + b * bstride + r, with off(a) = box_mult * a (expansion
// arrays) or start[a] (point arrays in sorted order).
// a load the scalar unit serves: the address is uniform across the wave and
// the array is read-only while the kernel runs
__device__ inline int ld_uniform(const int32_t *p, int i) {
    return ((const __attribute__((address_space(4))) int32_t *)p)[i];
}

// Column (box a, density d) of an array starts at off(a) + d bstride, its
// element k kstride further on (kstride > 1 only for k_fixed_apply inputs:
// the density-fastest charges, with start[] scaled by smult)
struct ColAddr {
    int64_t bstride;
    int64_t box_mult;
    const int32_t *start;
    int64_t smult = 1;
    int64_t kstride = 1;
    __device__ inline int64_t off(int a) const { return start ? (int64_t)start[a] * smult : box_mult * (int64_t)a; }
    // the same for a box index that is uniform across the wave
    __device__ inline int64_t off_u(int a) const {
        return start ? (int64_t)ld_uniform(start, a) * smult : box_mult * (int64_t)a;
    }
};

template <class TM>
struct Mfma;

// v_mfma_f64_16x16x4: result element i of lane l is D[4i + l/16][l%16]
template <>
struct Mfma<double> {
    typedef v4d acc_t;
    static __device__ inline acc_t zero() { return (v4d){0.0, 0.0, 0.0, 0.0}; }
    static __device__ inline acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int i, int g) { return 4 * i + g; }
    static __device__ inline int item_of(int r16) { return r16 >> 2; }
    static __device__ inline int group_of(int r16) { return r16 & 3; }
};

// v_mfma_f32_16x16x4: result element i of lane l is D[4(l/16) + i][l%16]
template <>
struct Mfma<float> {
    typedef v4f acc_t;
    static __device__ inline acc_t zero() { return (v4f){0.f, 0.f, 0.f, 0.f}; }
    static __device__ inline acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int i, int g) { return 4 * g + i; }
    static __device__ inline int item_of(int r16) { return r16 & 3; }
    static __device__ inline int group_of(int r16) { return r16 >> 2; }
};

struct TranslateArgs {
    const int32_t *cols_box;  // box of column group c / nbatch
    int ncols;                // number of (box, density) columns
    int nbatch;
    const int32_t *slots;     // [box][nops] source box or -1
    int nops;
    ColAddr in, out;
    int nrows_out;            // rows written per output column
    int logrow;               // >= 0: row holding sum Re A_0 (M2L); -1 otherwise
    const int32_t *level;
    const double *logside;
    // optional: operators present in 16-column tile t, tile_ops[tile_ptr[t] ..
    // tile_ptr[t+1]) (k_translate_split only; null = scan all nops slots)
    const int32_t *tile_ptr = nullptr;
    const int32_t *tile_ops = nullptr;
    const int32_t *tile_order = nullptr;  // optional launch order of the tiles (most operators first)
    const void *zero_col = nullptr;       // zeros of the input type, at least 4 S long (absent sources)
    const int32_t *xinit = nullptr;       // optional [box] nonzero: add to the output column (k_translate_split)
    int in_zero = 0;                      // k_tables_ct with density-fastest charges: point index of a zero block
};


// TI/TO: element types of input/output columns; TM: matrix-core type;
// RB: 16-row blocks of the output; S: 4-row steps of the input;
// SPLIT: add the A_lo product; ACCUM: out += instead of out =;
// LDSA: stage operators in LDS (off for very large operators).
template <class TI, class TO, class TM, int RB, int S, bool SPLIT, bool ACCUM, bool LDSA>
__global__ void __launch_bounds__(256) k_translate(TranslateArgs a, const TM *__restrict__ Ahi,
                                                   const TM *__restrict__ Alo, const TI *__restrict__ in,
                                                   TO *__restrict__ out) {
    typedef Mfma<TM> M;
    constexpr int AE = RB * S * 64;
    extern __shared__ unsigned char smem[];
    TM *sA = reinterpret_cast<TM *>(smem);
    TM *sAlo = sA + AE;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cl = lane & 15, g = lane >> 4;
    const int col = (blockIdx.x * 4 + wave) * 16 + cl;
    const bool valid = col < a.ncols;
    const int box = valid ? a.cols_box[col / a.nbatch] : 0;
    const int bt = valid ? col % a.nbatch : 0;
    typename M::acc_t acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = M::zero();
    for (int o = 0; o < a.nops; ++o) {
        const int src = valid ? a.slots[(int64_t)box * a.nops + o] : -1;
        if (!__syncthreads_or(src >= 0)) continue;
        const TM *Ao = Ahi + (int64_t)o * AE;
        const TM *Alo_o = SPLIT ? Alo + (int64_t)o * AE : nullptr;
        if (LDSA) {
            for (int e = tid; e < AE; e += 256) {
                sA[e] = Ao[e];
                if (SPLIT) sAlo[e] = Alo_o[e];
            }
            __syncthreads();
        }
        if (__ballot(src >= 0) != 0ull) {
            TM bv[S];
            const TI *ip = in + (src >= 0 ? a.in.off(src) + (int64_t)bt * a.in.bstride : 0) + g;
#pragma unroll
            for (int s = 0; s < S; ++s) bv[s] = (src >= 0) ? (TM)ip[4 * s] : (TM)0;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const int e = (r * S + s) * 64 + lane;
                    const TM av = LDSA ? sA[e] : Ao[e];
                    acc[r] = M::op(av, bv[s], acc[r]);
                    if (SPLIT) acc[r] = M::op(LDSA ? sAlo[e] : Alo_o[e], bv[s], acc[r]);
                }
            }
        }
        if (LDSA) __syncthreads();
    }
    double vals[RB][4];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) vals[r][i] = (double)acc[r][i];
    if (a.logrow >= 0) {
        // add A_0 log s (level of the target box) to row 0; clear the sum row
        const int rb2 = a.logrow >> 4, r16 = a.logrow & 15;
        const int i2 = M::item_of(r16), g2 = M::group_of(r16);
        double s0 = 0.0;
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (r == rb2 && i == i2) s0 = vals[r][i];
        s0 = __shfl(s0, g2 * 16 + cl, 64);
        if (g == M::group_of(0) && valid) vals[0][M::item_of(0)] += s0 * a.logside[a.level[box]];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (r == rb2 && i == i2 && g == g2) vals[r][i] = 0.0;
    }
    if (valid) {
        TO *op = out + a.out.off(box) + (int64_t)bt * a.out.bstride;
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = r * 16 + M::row(i, g);
                if (row < a.nrows_out) {
                    if (ACCUM) op[row] += (TO)vals[r][i];
                    else op[row] = (TO)vals[r][i];
                }
            }
    }
}

// Fixed-matrix variant for the pattern L2P launch (few columns, latency
// bound, at the end of an evaluation): a workgroup owns ONE 16-column tile and each of its waves
// one 16-row block of the output (blockDim = 64 x output row blocks), so a
// launch has four times the waves of k_translate and each wave's chain is
// one quarter of the operator.  The wave reads its operator rows straight
// from L2 together with the tile's input columns (an absent source reads
// the zero column), then runs S products.  Columns whose slot o is empty
// get exact zeros from that operator, so the per-column sum is the same as
// in k_translate.
template <class TI, class TO, class TM, int S, bool ACCUM>
__global__ void __launch_bounds__(256) k_pattern_op(TranslateArgs a, const TM *__restrict__ A,
                                                    const TI *__restrict__ in, TO *__restrict__ out) {
    typedef Mfma<TM> M;
    const int tid = threadIdx.x, lane = tid & 63, r = tid >> 6, nrb = blockDim.x >> 6;
    const int cl = lane & 15, g = lane >> 4;
    const int col = blockIdx.x * 16 + cl;
    const bool valid = col < a.ncols;
    const int box = valid ? a.cols_box[col / a.nbatch] : 0;
    const int bt = valid ? col % a.nbatch : 0;
    const TI *zc = static_cast<const TI *>(a.zero_col);
    const int64_t AE = (int64_t)nrb * S * 64;
    typename M::acc_t acc = M::zero();
    for (int o = 0; o < a.nops; ++o) {
        const int src = valid ? a.slots[(int64_t)box * a.nops + o] : -1;
        if (__ballot(src >= 0) == 0ull) continue;  // the same for every wave of the tile
        const TM *Ao = A + o * AE + (int64_t)r * S * 64 + lane;
        const TI *ip = (src >= 0 ? in + a.in.off(src) + (int64_t)bt * a.in.bstride : zc) + g;
        TM av[S], bv[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            av[s] = Ao[s * 64];
            bv[s] = (TM)ip[4 * s];
        }
#pragma unroll
        for (int s = 0; s < S; ++s) acc = M::op(av[s], bv[s], acc);
    }
    if (valid) {
        TO *op = out + a.out.off(box) + (int64_t)bt * a.out.bstride;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = r * 16 + M::row(i, g);
            if (row < a.nrows_out) {
                if (ACCUM) op[row] += (TO)acc[i];
                else op[row] = (TO)acc[i];
            }
        }
    }
}

// One fixed operator applied to many columns: out[:, c] (+)= A in[:, c]
// (pattern P2M of leaves, pattern L2P).  A has RB 16-row blocks and S 4-row
// input steps (A-fragment order).  Every wave keeps the whole operator in
// registers for the launch and owns one 16-column tile at a time, walking
// the tiles with a grid stride; it loads the next tile's input fragments
// before the products of the current one, so the loads are in flight while
// the matrix cores work.  Nothing is staged in LDS and there are no
// barriers.  The products are formed transposed, D^T = in^T A^T (the input
// fragments as the first matrix-core operand, the operator fragments, whose
// A-fragment order is the B-fragment order of A^T, as the second), so that
// a lane's results are one output row of four columns and a store
// instruction writes 16 consecutive rows of four columns instead of four
// rows of sixteen.  Each column's products still run s = 0 .. S-1 from zero
// per row block.  The clamped last column stands in for columns past the
// end (no branch around the loads); they store nothing.
// addflag (optional): columns of boxes with addflag[box] != 0 add even
// without ACCUM.  FIN (pattern L2P of a forward evaluation whose far field
// has no other writer): the column's value v at sorted target t goes to the
// output in user order, u[b][perm[t]] = (near[b][t] + v) + u[b][perm[t]]
// (u holds the correction row; without fin.add_u, u = near + v), the sum
// k_add_acc forms otherwise.
struct FinishArgs {
    const double *near = nullptr;  // [nbatch][ntgt] near-field sums, sorted order
    const int32_t *perm = nullptr; // sorted target -> user index
    int64_t m = 0;                 // output row length
    double *u = nullptr;
    bool add_u = true;             // add the correction rows already in u (false: u is only written)
};

// ALDS: the operator sits in LDS, copied once per workgroup, instead of in
// every wave's registers -- fewer registers, more waves per SIMD and so more
// loads in flight (the loads, not the products, bound these launches).
template <class TI, class TO, class TM, int RB, int S, bool ACCUM, bool FIN, bool ALDS>
__global__ void __launch_bounds__(256, ALDS ? 3 : 1) k_fixed_apply(const int32_t *__restrict__ cols_box, int ncols,
                                                                   int nbatch, ColAddr ia, ColAddr oa, int nrows_out,
                                                                   const TM *__restrict__ A,
                                                                   const TI *__restrict__ in, TO *__restrict__ out,
                                                                   const int32_t *__restrict__ addflag,
                                                                   FinishArgs fin) {
    typedef Mfma<TM> M;
    constexpr int AE = RB * S * 64;
    const int lane = threadIdx.x & 63;
    const int cl = lane & 15, g = lane >> 4;
    __shared__ TM sA[ALDS ? AE : 1];
    TM av[ALDS ? 1 : RB][ALDS ? 1 : S];
    if constexpr (ALDS) {
        for (int e = threadIdx.x; e < AE; e += blockDim.x) sA[e] = A[e];
        __syncthreads();
    } else {
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int s = 0; s < S; ++s) av[r][s] = A[(r * S + s) * 64 + lane];
    }
    const int ntiles = (ncols + 15) / 16;
    const int tstride = gridDim.x * (blockDim.x >> 6);
    // with nbatch a multiple of 16 a tile is one box's 16 densities: its box
    // and column start come through the scalar unit (no dependent vector
    // loads ahead of the column loads)
    const bool one_box = nbatch % 16 == 0;
    auto load = [&](int t, TM *bv) {
        const TI *ip;
        if (one_box) {
            const int box = ld_uniform(cols_box, t * 16 / nbatch);
            ip = in + ia.off_u(box) + (int64_t)(t * 16 % nbatch + cl) * ia.bstride + g * ia.kstride;
        } else {
            const int col = min(t * 16 + cl, ncols - 1);
            const int box = cols_box[col / nbatch], bt = col % nbatch;
            ip = in + ia.off(box) + (int64_t)bt * ia.bstride + g * ia.kstride;
        }
#pragma unroll
        for (int s = 0; s < S; ++s) bv[s] = (TM)ip[4 * s * ia.kstride];
    };
    int t = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    TM bcur[S], bnext[S];
    load(min(t, ntiles - 1), bcur);
    for (; t < ntiles; t += tstride) {
        load(min(t + tstride, ntiles - 1), bnext);
        typename M::acc_t accs[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) accs[r] = M::zero();
        // per k-step the RB operator fragments, then the RB products (with the
        // operator in LDS a scheduling barrier per step keeps the compiler from
        // loading all of it into registers ahead of the products)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            TM a_s[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                if constexpr (ALDS) a_s[r] = sA[(r * S + s) * 64 + lane];
                else a_s[r] = av[r][s];
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) accs[r] = M::op(bcur[s], a_s[r], accs[r]);
            if constexpr (ALDS) __builtin_amdgcn_sched_barrier(0);
        }
        // element i of a lane: output row r * 16 + cl of tile column M::row(i, g)
        if (FIN && one_box) {
            // one box per tile: its target rows and their permutation once for
            // all sixteen densities (the general path below reloads them per column)
            const int box = ld_uniform(cols_box, t * 16 / nbatch);
            const int64_t t0 = oa.off_u(box);
            int pr[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int row = r * 16 + cl;
                pr[r] = row < nrows_out ? fin.perm[t0 + row] : 0;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int bt = (t * 16 + M::row(i, g)) % nbatch;
                const double *nr = fin.near + (int64_t)bt * oa.bstride + t0;
                double *ub = fin.u + (int64_t)bt * fin.m;
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const int row = r * 16 + cl;
                    if (row < nrows_out) {
                        double *o = ub + pr[r];
                        *o = fin.add_u ? (nr[row] + (double)accs[r][i]) + *o : nr[row] + (double)accs[r][i];
                    }
                }
            }
        } else if (!FIN && one_box) {
            const int box = ld_uniform(cols_box, t * 16 / nbatch);
            const int64_t t0 = oa.off_u(box);
            const bool add = ACCUM || (addflag && ld_uniform(addflag, box));
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                TO *op = out + t0 + (int64_t)(t * 16 % nbatch + M::row(i, g)) * oa.bstride;
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const int row = r * 16 + cl;
                    if (row < nrows_out) {
                        if (add) op[row] += (TO)accs[r][i];
                        else op[row] = (TO)accs[r][i];
                    }
                }
            }
        } else
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int col = t * 16 + M::row(i, g);
            if (col >= ncols) continue;
            const int box = cols_box[col / nbatch], bt = col % nbatch;
            const int64_t t0 = oa.off(box), nb0 = (int64_t)bt * oa.bstride;
            if (FIN) {
                double *ub = fin.u + (int64_t)bt * fin.m;
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const int row = r * 16 + cl;
                    if (row < nrows_out) {
                        double *o = ub + fin.perm[t0 + row];
                        const double v = fin.near[nb0 + t0 + row] + (double)accs[r][i];
                        *o = fin.add_u ? v + *o : v;
                    }
                }
            } else {
                TO *op = out + t0 + nb0;
                const bool add = ACCUM || (addflag && addflag[box]);
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    const int row = r * 16 + cl;
                    if (row < nrows_out) {
                        if (add) op[row] += (TO)accs[r][i];
                        else op[row] = (TO)accs[r][i];
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) bcur[s] = bnext[s];
    }
}

// Pattern L2P of a uniform tree's deepest level, each leaf's local expansion
// taken together with its parent's through the class matrix B_q = L2P x L2L_q
// (so the L2L into that level never runs), and the finish of a forward
// evaluation: u[b][perm[t]] = (near[b][t] + v) + u[b][perm[t]] for the leaf's
// targets t.  A tile is one box's 16 densities from a.rec (grouped by child
// class, in tree order within a class); each workgroup serves one class, with
// the L2P and that class's B_q in LDS, and walks its class's tiles with a grid
// stride, one per wave.  The
// operators are in k-major fragments (lane group g takes the S consecutive
// expansion rows S g ..), so a lane's column elements are contiguous and load
// 16 bytes at a time.  The next tile's columns load while this tile's products
// run; this tile's parent columns and permutation load at its start, its near
// sums and output rows after the first product, all before they are needed.
// Every leaf has RB * 16 targets (the patterns are 16, 32 or 64 points).
struct L2PFinArgs {
    const int32_t *rec;    // [tile][4] {box, parent * 4 + class, first density, 0}
    int qbeg[5];           // class q's tiles: [qbeg[q], qbeg[q + 1])
    int64_t box_stride;    // local-expansion elements between boxes (nbatch PD)
    int PD;                // between the densities of a box
    const int32_t *tb;     // [box] first sorted target
    const double *near;    // [nbatch][ntgt], sorted order
    int64_t ntgt;
    const int32_t *perm;   // sorted target -> user index
    double *u;             // [nbatch][m], user order
    int64_t m;
};

// ADDU: add the correction rows already in u (else u is only written)
template <int RB, int S, bool ADDU>
__global__ void __launch_bounds__(256, 2) k_l2p_fin(L2PFinArgs a, const double *__restrict__ A,
                                                    const double *__restrict__ Bq4, const double *__restrict__ L) {
    typedef Mfma<double> M;
    constexpr int AE = RB * S * 64;
    static_assert(S % 2 == 0, "column elements load in pairs");
    __shared__ __align__(16) double sA[AE];
    __shared__ __align__(16) double sB[AE];
    // workgroup b runs on XCD b % 8: the four classes of one position are
    // workgroups b, b + 8, b + 16, b + 24, one XCD, so a parent's columns
    // (read by its four children, one per class) come from that XCD's L2
    // after the first read (the grid is a multiple of 32)
    const int q = (blockIdx.x >> 3) & 3;
    const int pos = (blockIdx.x & 7) | ((blockIdx.x >> 5) << 3);
    const int lane = threadIdx.x & 63, cl = lane & 15, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int e = threadIdx.x; e < AE; e += 256) {
        sA[e] = A[e];
        sB[e] = Bq4[(int64_t)q * AE + e];
    }
    __syncthreads();
    const int jq = a.qbeg[q], nq = a.qbeg[q + 1] - jq;
    const int stride = (int)gridDim.x;  // waves of this class: a quarter of the workgroups, four waves each
    int j = pos * 4 + wave;
    if (j >= nq) return;
    const int32_t *rec = a.rec + (int64_t)jq * 4;
    // Addresses: a uniform base (scalar registers) plus a 32-bit lane offset,
    // most of them fixed for the launch (the host checks that the offsets fit).
    // Elements S g .. S g + S - 1 of density column d + cl of box b:
    const unsigned col_off = (unsigned)(cl * a.PD + S * g) * 8u;
    auto ld_cols = [&](int b, int d, double(&x)[S]) {
        const char *base = reinterpret_cast<const char *>(L + (int64_t)b * a.box_stride + (int64_t)d * a.PD);
#pragma unroll
        for (int s = 0; s < S; s += 2) {
            const double2 v = *reinterpret_cast<const double2 *>(base + (size_t)col_off + (size_t)(s * 8));
            x[s] = v.x;
            x[s + 1] = v.y;
        }
    };
    // near sums and output rows of result element (r, i): density d0 + 4 i + g
    // (M::row(i, g)), target row r * 16 + cl
    const unsigned near_off0 = (unsigned)(g * a.ntgt + cl) * 8u;
    // (a scheduling barrier per k-step keeps the compiler from reading the
    // whole operator into registers ahead of the products)
    auto product = [&](const double(&x)[S], const double *op, typename M::acc_t(&acc)[RB], unsigned oaddr) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int r = 0; r < RB; ++r)
                acc[r] = M::op(x[s], *reinterpret_cast<const double *>(reinterpret_cast<const char *>(op) + oaddr +
                                                                      (r * S + s) * 64 * 8),
                               acc[r]);
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    unsigned oaddr = (unsigned)lane * 8u;
    int box = ld_uniform(rec, 4 * j), pcv = ld_uniform(rec, 4 * j + 1), d0 = ld_uniform(rec, 4 * j + 2);
    double xa[S];
    ld_cols(box, d0, xa);
    for (; j < nq; j += stride) {
        const int jn = j + stride < nq ? j + stride : j;
        const int boxn = ld_uniform(rec, 4 * jn), pcn = ld_uniform(rec, 4 * jn + 1), dn = ld_uniform(rec, 4 * jn + 2);
        const int t0 = ld_uniform(a.tb, box);
        // issue order (loads complete in order): this tile's parent columns and
        // permutation, then the next tile's own columns
        double xp[S], xn[S];
        ld_cols(pcv >> 2, d0, xp);
        unsigned uoff[RB];
        {
            const char *pb = reinterpret_cast<const char *>(a.perm + t0);
#pragma unroll
            for (int r = 0; r < RB; ++r)
                uoff[r] = (unsigned)(g * a.m + *reinterpret_cast<const int32_t *>(pb + (size_t)((r * 16 + cl) * 4))) * 8u;
        }
        ld_cols(boxn, dn, xn);
        __builtin_amdgcn_sched_barrier(0);
        typename M::acc_t acc[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[r] = M::zero();
        product(xa, sA, acc, oaddr);
        __builtin_amdgcn_sched_barrier(0);
        double nv[RB][4], uv[RB][4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const char *nb = reinterpret_cast<const char *>(a.near + (int64_t)(d0 + 4 * i) * a.ntgt + t0);
            const char *ub = reinterpret_cast<const char *>(a.u + (int64_t)(d0 + 4 * i) * a.m);
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                nv[r][i] = *reinterpret_cast<const double *>(nb + (size_t)near_off0 + (size_t)(r * 16 * 8));
                uv[r][i] = ADDU ? *reinterpret_cast<const double *>(ub + (size_t)uoff[r]) : 0.0;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        product(xp, sB, acc, oaddr);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            char *ub = reinterpret_cast<char *>(a.u + (int64_t)(d0 + 4 * i) * a.m);
#pragma unroll
            for (int r = 0; r < RB; ++r)
                *reinterpret_cast<double *>(ub + (size_t)uoff[r]) =
                    ADDU ? (nv[r][i] + acc[r][i]) + uv[r][i] : nv[r][i] + acc[r][i];
        }
        // the operator fragments are read from LDS per tile (hoisted out of
        // the loop they would need every register)
        asm volatile("" : "+v"(oaddr));
#pragma unroll
        for (int s = 0; s < S; ++s) xa[s] = xn[s];
        box = boxn;
        pcv = pcn;
        d0 = dn;
    }
}

// Split-operator variant for the large M2L launch and the near tables: the
// NW waves of a workgroup (4 by default, 2 when the plan's autotuner finds
// that faster) share ONE 16-column tile and take every NW-th active operator,
// reading operator fragments straight from L2 (no barriers in the main
// loop, four times more waves in flight); their partial tiles are summed
// through LDS in a fixed order at the end.
template <class TI, class TO, class TM, int RB, int S, bool SPLIT, bool ACCUM, int NW = 4>
__global__ void __launch_bounds__(64 * NW) k_translate_split(TranslateArgs a, const TM *__restrict__ Ahi,
                                                         const TM *__restrict__ Alo,
                                                         const TI *__restrict__ in, TO *__restrict__ out) {
    typedef Mfma<TM> M;
    constexpr int AE = RB * S * 64;
    static_assert(NW == 2 || NW == 4, "two or four waves per tile");
    constexpr int NT = 64 * NW;
    __shared__ double red[NW - 1][RB * 4][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cl = lane & 15, g = lane >> 4;
    const int tile = a.tile_order ? a.tile_order[blockIdx.x] : (int)blockIdx.x;
    const int col = tile * 16 + cl;
    const bool valid = col < a.ncols;
    const int box = valid ? a.cols_box[col / a.nbatch] : 0;
    const int bt = valid ? col % a.nbatch : 0;
    typename M::acc_t acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = M::zero();
    const TI *zc = static_cast<const TI *>(a.zero_col);
    auto product = [&](int o, int src) {
        // an absent source reads the zero column: no branch around the loads
        const TI *ip = (src >= 0 ? in + a.in.off(src) + (int64_t)bt * a.in.bstride : zc) + g;
        TM bv[S];
#pragma unroll
        for (int s = 0; s < S; ++s) bv[s] = (TM)ip[4 * s];
        const TM *Ao = Ahi + (int64_t)o * AE + lane;
        const TM *Alo_o = SPLIT ? Alo + (int64_t)o * AE + lane : nullptr;
        // operator fragments one 16-row block at a time: the loads of block
        // r + 1 are in flight while block r is on the matrix cores (the
        // scheduling barriers keep the compiler from pairing every load with
        // its product and a full wait)
        TM ah[2][S], al[2][SPLIT ? S : 1];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            ah[0][s] = Ao[s * 64];
            if (SPLIT) al[0][s] = Alo_o[s * 64];
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int c = r & 1;
            if (r + 1 < RB) {
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    ah[c ^ 1][s] = Ao[((r + 1) * S + s) * 64];
                    if (SPLIT) al[c ^ 1][s] = Alo_o[((r + 1) * S + s) * 64];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                acc[r] = M::op(ah[c][s], bv[s], acc[r]);
                if (SPLIT) acc[r] = M::op(al[c][s], bv[s], acc[r]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    };
    if (a.tile_ptr) {
        // the tile's operators and each column's source per operator, staged in
        // LDS 64 operators at a time (no dependent global loads in the loop)
        __shared__ int32_t s_ops[64];
        __shared__ int32_t s_src[64][16];
        const int e0 = a.tile_ptr[tile], nt = a.tile_ptr[tile + 1] - e0;
        for (int c0 = 0; c0 < nt; c0 += 64) {
            const int nc = min(64, nt - c0);
            __syncthreads();
            for (int i = tid; i < nc; i += NT) s_ops[i] = a.tile_ops[e0 + c0 + i];
            __syncthreads();
            for (int i = tid; i < nc * 16; i += NT) {
                const int oi = i >> 4, c = i & 15, cc = tile * 16 + c;
                s_src[oi][c] = cc < a.ncols ? a.slots[(int64_t)a.cols_box[cc / a.nbatch] * a.nops + s_ops[oi]] : -1;
            }
            __syncthreads();
            for (int e = wave; e < nc; e += NW) product(s_ops[e], s_src[e][cl]);
        }
    } else {
        int it = 0;  // index among the tile's active operators
        for (int o = 0; o < a.nops; ++o) {
            const int src = valid ? a.slots[(int64_t)box * a.nops + o] : -1;
            if (__ballot(src >= 0) == 0ull) continue;
            const bool mine = it % NW == wave;
            ++it;
            if (mine) product(o, src);
        }
    }
    // fixed-order sum of the partial tiles: wave 0 + 1 + ... + NW-1
    if (wave > 0) {
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) red[wave - 1][r * 4 + i][lane] = (double)acc[r][i];
    }
    __syncthreads();
    if (wave != 0) return;
    double vals[RB][4];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            vals[r][i] = (double)acc[r][i];
#pragma unroll
            for (int v = 0; v < NW - 1; ++v) vals[r][i] += red[v][r * 4 + i][lane];
        }
    if (a.logrow >= 0) {
        const int rb2 = a.logrow >> 4, r16 = a.logrow & 15;
        const int i2 = M::item_of(r16), g2 = M::group_of(r16);
        double s0 = 0.0;
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (r == rb2 && i == i2) s0 = vals[r][i];
        s0 = __shfl(s0, g2 * 16 + cl, 64);
        if (g == M::group_of(0) && valid) vals[0][M::item_of(0)] += s0 * a.logside[a.level[box]];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (r == rb2 && i == i2 && g == g2) vals[r][i] = 0.0;
    }
    if (valid) {
        TO *op = out + a.out.off(box) + (int64_t)bt * a.out.bstride;
        const bool add = ACCUM || (a.xinit && a.xinit[box]);
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = r * 16 + M::row(i, g);
                if (row < a.nrows_out) {
                    if (add) op[row] += (TO)vals[r][i];
                    else op[row] = (TO)vals[r][i];
                }
            }
    }
}

// Near-field tables, one wave per workgroup over CT 16-column tiles at once.
// Every leaf of a table level applies the same NTOPS operators (one per
// neighbour slot), so the wave loads each operator fragment once and applies
// it to the CT tiles' source columns: CT times less operator traffic from L2
// than one tile per wave, which is what bounds the one-tile form (a 64 x 64
// FP64 operator per 16-column product asks L2 for more bytes per cycle than
// it delivers at the matrix cores' rate).  tile_ptr / tile_ops list the
// operators present in each group of 16 CT columns; absent sources read the
// zero column.  Stores (each table leaf's sums come from its one group).
// IL: the charges come density fastest, element (point k of box b, density
// d) at (start[b] + k) nbatch + d, so that a load of four points of sixteen
// densities is one contiguous 512-byte block (with one density per row the
// sixteen densities of a box lie a whole charge array apart).
//
// Schedule: k-steps outermost, so each step issues RB * CT independent
// products (no product waits on the one before it).  Operator fragments and
// source charges stream PF k-steps ahead of the products through two small
// register rings, across operator boundaries (the first steps of the next
// operator and of its source columns load during the last steps of this
// one); the rings leave room for three waves per SIMD.
//
// Addressing is kept off the VALU, which shares the SIMD with the FP64
// products: the operator code comes through the scalar unit, so an
// operator's fragments are one uniform base plus fixed per-lane offsets.  IL: each column's source is staged as a point offset into the
// charge copy (an absent source as the block of zeros at point a.in_zero),
// so a column address is one 24-bit multiply-add into a 32-bit byte offset;
// NB > 0 fixes nbatch (the k-step stride then folds into the load offsets).
template <int RB, int S, int CT, bool IL, int NB = 0>
__global__ void __launch_bounds__(64) k_tables_ct(TranslateArgs a, const double *__restrict__ A,
                                                  const double *__restrict__ in, double *__restrict__ out) {
    typedef Mfma<double> M;
    constexpr int AE = RB * S * 64;
    constexpr int W = 16 * CT;  // columns per group
    constexpr int PF = 3, NBUF = PF + 1;  // operator prefetch distance (k-steps), ring slots
    static_assert(S % NBUF == 0, "the ring wraps at operator boundaries");
    __shared__ int32_t s_ops[64];
    __shared__ int32_t s_src[64 + 1][W];  // one more entry: the look-ahead past the last operator
    const int lane = threadIdx.x, cl = lane & 15, g = lane >> 4;
    const int tile = ld_uniform(a.tile_order, blockIdx.x);
    const int nbatch = NB > 0 ? NB : a.nbatch;
    int box[CT], bt[CT];
    bool valid[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        const int col = tile * W + c * 16 + cl;
        valid[c] = col < a.ncols;
        box[c] = valid[c] ? a.cols_box[col / nbatch] : 0;
        bt[c] = valid[c] ? col % nbatch : 0;
    }
    typename M::acc_t acc[CT][RB];
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[c][r] = M::zero();
    const double *zc = static_cast<const double *>(a.zero_col);
    // IL: element k = 4 s + g of column c of entry e is at byte
    // col_off(e, c) + s * kstb of the charge copy
    const char *inb = reinterpret_cast<const char *>(in);
    const unsigned nb8 = (unsigned)nbatch * 8u, kstb = 32u * (unsigned)nbatch;
    unsigned lc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) lc[c] = (unsigned)(g * nbatch + bt[c]) * 8u;
    // non-IL: element k = 4 s + g of a source column is at src_col(e, c)[4 s]
    auto src_col = [&](int e, int c) {
        const int src = s_src[e][c * 16 + cl];
        return (src >= 0 ? in + a.in.off(src) + (int64_t)bt[c] * a.in.bstride : zc) + g;
    };
    auto col_addr = [&](int e, unsigned(&off)[CT], const double *(&ip)[CT]) {
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            if constexpr (IL) off[c] = __umul24((unsigned)s_src[e][c * 16 + cl], nb8) + lc[c];
            else ip[c] = src_col(e, c);
        }
    };
    // operator fragment (row block r, k-step s) of the operator at byte base ab
    const unsigned lane8 = (unsigned)lane * 8u;
    auto ld_op = [&](const char *ab, int r, int s) {
        return *reinterpret_cast<const double *>(ab + (size_t)lane8 + (size_t)((r * S + s) * 64 * 8));
    };
    auto op_base = [&](int op) { return reinterpret_cast<const char *>(A + (int64_t)op * AE); };
    const int e0 = ld_uniform(a.tile_ptr, tile), nt = ld_uniform(a.tile_ptr, tile + 1) - e0;
    for (int c0 = 0; c0 < nt; c0 += 64) {
        const int nc = min(64, nt - c0);
        __syncthreads();
        for (int i = lane; i < nc; i += 64) s_ops[i] = a.tile_ops[e0 + c0 + i];
        __syncthreads();
        for (int i = lane; i < (nc + 1) * W; i += 64) {
            const int oi = i / W, c = i % W, cc = tile * W + c;
            const int src = cc < a.ncols && oi < nc ? a.slots[(int64_t)a.cols_box[cc / nbatch] * a.nops + s_ops[oi]]
                                                    : -1;
            if constexpr (IL) s_src[oi][c] = src >= 0 ? (int)a.in.off(src) : a.in_zero;
            else s_src[oi][c] = src;
        }
        __syncthreads();
        // rings: k-step j of the stream (operator fragments and source
        // charges alike) sits in slot j % NBUF, loaded PF steps ahead
        double af[NBUF][RB], cv[NBUF][CT];
        unsigned offc[CT], offn[CT];
        const double *ipc[CT], *ipn[CT];
        col_addr(0, offc, ipc);
        auto ld_ch = [&](int s, double(&dst)[CT], const unsigned(&off)[CT], const double *const(&ip)[CT]) {
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                if constexpr (IL) dst[c] = *reinterpret_cast<const double *>(inb + (size_t)off[c] + (size_t)s * kstb);
                else dst[c] = ip[c][4 * s];
            }
        };
        {
            const char *A0 = op_base(ld_uniform(a.tile_ops, e0 + c0));
#pragma unroll
            for (int p = 0; p < PF; ++p) {
#pragma unroll
                for (int r = 0; r < RB; ++r) af[p][r] = ld_op(A0, r, p);
                ld_ch(p, cv[p], offc, ipc);
            }
        }
        for (int e = 0; e < nc; ++e) {
            // this operator and the next (this one again after the last: loaded, never used)
            const char *Ao = op_base(ld_uniform(a.tile_ops, e0 + c0 + e));
            const char *An = op_base(ld_uniform(a.tile_ops, e0 + c0 + (e + 1 < nc ? e + 1 : e)));
            col_addr(e + 1, offn, ipn);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int sp = s + PF;
#pragma unroll
                for (int r = 0; r < RB; ++r) af[sp % NBUF][r] = sp < S ? ld_op(Ao, r, sp) : ld_op(An, r, sp - S);
                if (sp < S) ld_ch(sp, cv[sp % NBUF], offc, ipc);
                else ld_ch(sp - S, cv[sp % NBUF], offn, ipn);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int c = 0; c < CT; ++c) acc[c][r] = M::op(af[s % NBUF][r], cv[s % NBUF][c], acc[c][r]);
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                offc[c] = offn[c];
                ipc[c] = ipn[c];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CT; ++c) {
        if (!valid[c]) continue;
        double *op = out + a.out.off(box[c]) + (int64_t)bt[c] * a.out.bstride;
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = r * 16 + M::row(i, g);
                if (row < a.nrows_out) op[row] = acc[c][r][i];
            }
    }
}

// Dynamic LDS bytes of a k_translate launch (0 when operators stay in global memory).
template <class TM, int RB, int S, bool SPLIT>
constexpr size_t translate_lds_bytes() {
    return (size_t)(SPLIT ? 2 : 1) * RB * S * 64 * sizeof(TM);
}
template <class TM, int RB, int S, bool SPLIT>
constexpr bool translate_ldsa() {
    return translate_lds_bytes<TM, RB, S, SPLIT>() <= 61440;
}

}  // namespace vp

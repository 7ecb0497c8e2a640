// M2L in diagonally scaled form on matrix cores.
//
// With the side-scaled expansions of this library the M2L operator for a
// source box at (target centre + s t) factors as
//     B_0 = A_0 (log s + log(-t)) + sum_{k>=1} y_k
//     B_l = t^-l [ -A_0 / l + sum_{k>=1} C(l+k-1, k-1) y_k ],   l >= 1
// with y_k = (-t)^-k A_k: a complex diagonal scaling of the source column,
// ONE real matrix Q (Q[0][k] = 1, Q[l][0] = -1/l, Q[l][k] = C(l+k-1, k-1),
// Q[0][0] = 0) that is the same for all 40 offsets, and a complex diagonal
// scaling of the result.  Since t^-l = (-1)^l (-t)^-l, the sign (-1)^l is
// folded into row l of Q (the matrix passed here), and the one table
// (-t)^-k serves both scalings.  Because Q is real it acts on the real and the
// imaginary parts separately: the contraction per translation is two real
// P x P products instead of one real 2P x 2P product, and no per-offset
// operator is read from memory.  The terms summed are the same products as
// in the unfactored operator (only their grouping differs), so the rounding
// behaviour is that of the plain operator.
//
// Work split: a 16-column tile (boxes x densities, grouped by child class
// so the tile shares its offsets) per workgroup; its NW waves (4 by default,
// 2 when the plan's autotuner finds that faster) take every NW-th offset
// present in the tile (listed at plan time, with each column's source box)
// and their partial sums are added through LDS in a fixed order.
// The diagonal scalings of all 40 offsets sit in LDS for the whole tile and
// the lane's Q fragments in registers; the loop has no branch around a load
// and no dependent global load, and at 166 registers three waves share each
// SIMD, so the other waves' products cover one wave's column loads.
#pragma once

#include "vp_translate.hpp"

namespace vp {

struct M2LScaledArgs {
    const int32_t *cols_box;  // box of column group c / nbatch
    int ncols;                // (box, density) columns
    int nbatch;
    const int32_t *tile_ptr;  // offsets present in 16-column tile t: tile_ops[tile_ptr[t] .. tile_ptr[t+1])
    const int32_t *tile_ops;
    const int32_t *tile_src;  // [tile op][16]: source box of each column of the tile, or -1
    const int32_t *tile_order;  // launch order of the tiles (most offsets first; k_m2l_wave: in groups of four)
    int P;                    // complex coefficients per expansion
    int64_t box_stride;       // elements between the columns of consecutive boxes
    int64_t bt_stride;        // elements between the densities of one box
    int PD;                   // rows per column (re 0..P-1, im P..2P-1, zero padding)
    const int32_t *level;
    const double *logside;    // log of the box side per level
    const void *zero_col;     // PD zeros of the input type (the column of an absent source)
    const int32_t *xinit;     // [box] nonzero: the output column already holds P2L terms; add to it
    int zero_box;             // k_m2l_wave: box index of an all-zero block of the input array
};


// Column of one source for the k-steps of lane group g (k = g*S + s).  An
// absent source reads a column of zeros.  Rows k >= P of the real part (the
// first imaginary coefficients) and of the imaginary part (zero padding; the
// column has at least P + PQ rows) are read as they are: the zero rows
// k >= P of the input scaling remove them.  Every lane loads from one base
// address with constant offsets; no load sits behind a branch.
template <class TI, class TM, int S>
__device__ inline void m2l_load_col(const TI *__restrict__ ip, int g, int P, TM (&xr)[S], TM (&xi)[S]) {
    const TI *pr = ip + g * S, *pi = ip + P + g * S;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        xr[s] = (TM)pr[s];
        xi[s] = (TM)pi[s];
    }
}

// Q in A-fragment order [rb][s][lane] for k = 4 s + lane/16 (regathered here
// for k = (lane/16) S + s), rows multiplied by (-1)^l; tin [NOFF][RB*16][2]
// (re, im) = (-t)^-k, the input and (with Q's row signs) the output scaling;
// logt [NOFF][2] = log(-t).
template <class TI, class TO, class TM, int RB, int NW = 4>
__global__ void __launch_bounds__(64 * NW, 12 / NW) k_m2l_scaled(M2LScaledArgs a, const TM *__restrict__ Qf,
                                                    const TM *__restrict__ tin,
                                                    const double *__restrict__ logt, const TI *__restrict__ in,
                                                    TO *__restrict__ out) {
    typedef Mfma<TM> M;
    constexpr int S = RB * 4;  // k-steps: lane group g takes k = g*S + s
    constexpr int PQ = RB * 16;
    constexpr int NR = RB * 4 * 2 + 2;  // reduced values per lane: B re/im per item, A_0 sum re/im
    constexpr int TAB = NOFF * PQ * 2;  // elements of one scaling table
    constexpr int TBYTES = TAB * (int)sizeof(TM) + NOFF * 2 * (int)sizeof(double);
    static_assert(NW == 2 || NW == 4, "two or four waves per tile");
    constexpr int NT = 64 * NW;  // threads
    constexpr int RBYTES = (NW - 1) * NR * 64 * (int)sizeof(double);
    // scaling tables during the loop, the cross-wave partial sums after it
    __shared__ __align__(16) unsigned char s_raw[TBYTES > RBYTES ? TBYTES : RBYTES];
    __shared__ int32_t s_ops[NOFF];
    __shared__ int32_t s_src[NOFF][16];
    TM *s_tin = reinterpret_cast<TM *>(s_raw);
    double *s_logt = reinterpret_cast<double *>(s_raw + TAB * sizeof(TM));
    double(*red)[NR][64] = reinterpret_cast<double(*)[NR][64]>(s_raw);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cl = lane & 15, g = lane >> 4;
    const int tile = a.tile_order[blockIdx.x];
    const int col = tile * 16 + cl;
    const bool valid = col < a.ncols;
    const int box = valid ? a.cols_box[col / a.nbatch] : 0;
    const int bt = valid ? col % a.nbatch : 0;
    const int P = a.P;

    // stage the tile's offsets and sources and the tables of all offsets
    const int e0 = a.tile_ptr[tile], nt = a.tile_ptr[tile + 1] - e0;
    for (int i = tid; i < nt; i += NT) s_ops[i] = a.tile_ops[e0 + i];
    for (int i = tid; i < nt * 16; i += NT) s_src[i >> 4][i & 15] = a.tile_src[(int64_t)e0 * 16 + i];
    {
        constexpr int CH = TAB * (int)sizeof(TM) / 16;  // 16-byte chunks per table
        const uint4 *gi = reinterpret_cast<const uint4 *>(tin);
        uint4 *si = reinterpret_cast<uint4 *>(s_tin);
        for (int i = tid; i < CH; i += NT) si[i] = gi[i];
        if (tid < 2 * NOFF) s_logt[tid] = logt[tid];
    }
    TM q[RB][S];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int k = g * S + s;
            q[r][s] = Qf[(r * S + (k >> 2)) * 64 + (k & 3) * 16 + cl];
        }
    __syncthreads();

    double br[RB][4], bi[RB][4];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) br[r][i] = bi[r][i] = 0.0;
    double a0r = 0.0, a0i = 0.0;  // sum of A_0 over the sources (lanes g == 0)
    const int64_t bt_off = (int64_t)bt * a.bt_stride;

    // this wave's offsets: every NW-th one present in the tile
    int e = wave;
    const TI *zc = static_cast<const TI *>(a.zero_col);
    TM xr[S], xi[S];
    {
        const int src = e < nt ? s_src[e][cl] : -1;
        m2l_load_col<TI, TM, S>(src >= 0 ? in + (int64_t)src * a.box_stride + bt_off : zc, g, P, xr, xi);
    }
    const double m0 = g == 0 ? 1.0 : 0.0;  // lanes holding k = 0 at step 0
    for (; e < nt; e += NW) {
        const int o = s_ops[e];
        const TM *ti = s_tin + o * PQ * 2;
        {
            // A_0 log(-t): the offset-dependent part of the k = 0 column
            // (step 0 of lane group 0); other lanes add exact zeros
            const double x0r = (double)xr[0] * m0, x0i = (double)xi[0] * m0;
            const double lr = s_logt[2 * o], li = s_logt[2 * o + 1];
            br[0][M::item_of(0)] += x0r * lr - x0i * li;
            bi[0][M::item_of(0)] += x0r * li + x0i * lr;
            a0r += x0r;
            a0i += x0i;
        }
        // the next offset's source columns, into the registers the current
        // coefficients free once scaled (the compiler issues these loads at
        // the top of the next iteration, as eight 16-byte loads)
        const int en = e + NW;
        const int srcn = en < nt ? s_src[en][cl] : -1;
        const TI *ipn = srcn >= 0 ? in + (int64_t)srcn * a.box_stride + bt_off : zc;
        const TI *pnr = ipn + g * S, *pni = ipn + P + g * S;
        typename M::acc_t zr[RB], zi[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            zr[r] = M::zero();
            zi[r] = M::zero();
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int k = g * S + s;
            // input scaling y_k = (-t)^-k A_k, then the next offset's coefficient
            const TM wr = ti[2 * k], wi = ti[2 * k + 1];
            const TM yr = xr[s] * wr - xi[s] * wi;
            const TM yi = xr[s] * wi + xi[s] * wr;
            xr[s] = (TM)pnr[s];
            xi[s] = (TM)pni[s];
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const TM qv = q[r][s];
                zr[r] = M::op(qv, yr, zr[r]);
                zi[r] = M::op(qv, yi, zi[r]);
            }
        }
        const TM *to = ti;  // (-t)^-l; the sign (-1)^l is in Q
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int l = r * 16 + M::row(i, g);
                const double vr = (double)to[2 * l], vi = (double)to[2 * l + 1];
                const double zre = (double)zr[r][i], zim = (double)zi[r][i];
                br[r][i] += zre * vr - zim * vi;
                bi[r][i] += zre * vi + zim * vr;
            }
    }
    // fixed-order sum of the waves' partial results (the tables' LDS is
    // reused once every wave has left the loop)
    __syncthreads();
    if (wave > 0) {
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                red[wave - 1][(r * 4 + i) * 2][lane] = br[r][i];
                red[wave - 1][(r * 4 + i) * 2 + 1][lane] = bi[r][i];
            }
        red[wave - 1][NR - 2][lane] = a0r;
        red[wave - 1][NR - 1][lane] = a0i;
    }
    __syncthreads();
    if (wave != 0 || !valid) return;
    // wave 0 + 1 + ... + NW-1, left to right
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = (r * 4 + i) * 2;
#pragma unroll
            for (int v = 0; v < NW - 1; ++v) {
                br[r][i] += red[v][e][lane];
                bi[r][i] += red[v][e + 1][lane];
            }
        }
#pragma unroll
    for (int v = 0; v < NW - 1; ++v) {
        a0r += red[v][NR - 2][lane];
        a0i += red[v][NR - 1][lane];
    }
    if (g == 0) {
        const double ls = a.logside[a.level[box]];
        br[0][M::item_of(0)] += a0r * ls;
        bi[0][M::item_of(0)] += a0i * ls;
    }
    TO *op = out + (int64_t)box * a.box_stride + (int64_t)bt * a.bt_stride;
    const bool add = a.xinit[box] != 0;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int l = r * 16 + M::row(i, g);
            if (l < P) {
                op[l] = (TO)(add ? (double)op[l] + br[r][i] : br[r][i]);
                op[P + l] = (TO)(add ? (double)op[P + l] + bi[r][i] : bi[r][i]);
            }
        }
    for (int row = 2 * P + g; row < a.PD; row += 4) op[row] = (TO)0;
}

// One tile per wave: the workgroup's four waves take four tiles of the launch
// order (consecutive, so neighbouring boxes that share source columns run
// together) and each runs ALL of its tile's offsets.  No partial sums cross
// waves (no reduction through LDS, no barrier after the prologue, no wave
// idling on a short share of the offsets), and the scaling tables are staged
// once per four tiles.
//
// The loop is written for the lowest VALU count per offset: FP64 VALU
// instructions and FP64 matrix-core products share the SIMD's issue, so each
// VALU instruction in the loop takes time from the products.  Per offset it
// issues the two diagonal scalings (four FMAs per complex element, the output
// one accumulating), four FMAs and two additions for the A_0 log(-t) term and
// two integer operations: the offset code comes through the scalar unit, an
// absent source reads the all-zero column block at box index zero_box of the
// input array (so no select), the column address is one 24-bit multiply-add
// into a 32-bit offset from a uniform base, and log(-t) sits in the staged
// table beside the output rows where only lane group 0 (which holds row 0)
// reads a nonzero entry.  The input array must be under 4 GiB (checked by
// the launch).  The next offset's source columns load into a second register
// buffer at the start of each offset, a whole offset ahead of their use; Q's
// fragments come from LDS so the two buffers fit three waves per SIMD.
template <class TI, class TO, class TM, int RB>
__global__ void __launch_bounds__(256, 3) k_m2l_wave(M2LScaledArgs a, const TM *__restrict__ Qf,
                                                     const TM *__restrict__ tin, const double *__restrict__ logt,
                                                     const TI *__restrict__ in, TO *__restrict__ out) {
    typedef Mfma<TM> M;
    constexpr int S = RB * 4;
    constexpr int PQ = RB * 16;
    constexpr int ROWB = 2 * (int)sizeof(TM);                 // one (re, im) row of a table
    constexpr int GSTEP = sizeof(TM) == 8 ? ROWB : 4 * ROWB;  // output-row bytes between lane groups
    constexpr int OSTR = PQ * ROWB + 4 * GSTEP;               // one offset: PQ rows, then log(-t) per lane group
    __shared__ __align__(16) unsigned char s_tab[NOFF * OSTR];
    __shared__ int32_t s_src[4][NOFF + 1][16];
    __shared__ __align__(16) TM s_q[RB * S * 64];  // Q's A fragments [s][r][lane]

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int cl = lane & 15, g = lane >> 4;
    for (int i = tid; i < NOFF * PQ; i += 256) {
        const int o = i / PQ, k = i - o * PQ;
        TM *d = reinterpret_cast<TM *>(s_tab + o * OSTR + k * ROWB);
        d[0] = tin[2 * i];
        d[1] = tin[2 * i + 1];
    }
    for (int i = tid; i < NOFF * 4; i += 256) {
        const int o = i >> 2, gg = i & 3;
        double *d = reinterpret_cast<double *>(s_tab + o * OSTR + PQ * ROWB + gg * GSTEP);
        d[0] = gg == 0 ? logt[2 * o] : 0.0;
        d[1] = gg == 0 ? logt[2 * o + 1] : 0.0;
    }
    for (int i = tid; i < RB * S * 64; i += 256) {
        const int s = i / (RB * 64), r = (i / 64) % RB, l = i & 63;
        const int k = (l >> 4) * S + s;
        s_q[i] = Qf[(r * S + (k >> 2)) * 64 + (k & 3) * 16 + (l & 15)];
    }
    __syncthreads();
    const int ntiles = (a.ncols + 15) / 16;
    const int ti = blockIdx.x * 4 + wave;
    if (ti >= ntiles) return;
    const int tile = ld_uniform(a.tile_order, ti);
    const int e0 = ld_uniform(a.tile_ptr, tile), nt = ld_uniform(a.tile_ptr, tile + 1) - e0;
    const int col = tile * 16 + cl;
    const bool valid = col < a.ncols;
    const int box = valid ? a.cols_box[col / a.nbatch] : 0;
    const int bt = valid ? col % a.nbatch : 0;
    const int P = a.P;

    // each column's source per offset, absent ones as the zero block, and one
    // more entry (the zero block) read by the last offset's look-ahead
    for (int i = lane; i < (nt + 1) * 16; i += 64) {
        const int e = i >> 4;
        const int v = e < nt ? a.tile_src[(int64_t)(e0 + e) * 16 + (i & 15)] : -1;
        s_src[wave][e][i & 15] = v >= 0 ? v : a.zero_box;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    unsigned qaddr = (unsigned)lane * sizeof(TM);
    double br[RB][4], bi[RB][4];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) br[r][i] = bi[r][i] = 0.0;
    double a0r = 0.0, a0i = 0.0;  // sum of A_0 over the sources (used by lane group 0)
    // source column address: uniform base + box * box bytes + this lane's part
    const char *in_re = reinterpret_cast<const char *>(in);
    const char *in_im = reinterpret_cast<const char *>(in + P);
    const unsigned sbytes = (unsigned)(a.box_stride * (int64_t)sizeof(TI));
    const unsigned lconst = (unsigned)(((int64_t)bt * a.bt_stride + g * S) * (int64_t)sizeof(TI));
    const unsigned lin = (unsigned)(g * S * ROWB), lout = (unsigned)(g * GSTEP);
    // two column buffers: offset e computes from one while the other receives
    // offset e + 1's columns (the loop is unrolled by two, so the loads land
    // in place and stay in flight across the products)
    auto load = [&](int e, TM(&xr)[S], TM(&xi)[S]) {
        const unsigned off = __umul24((unsigned)s_src[wave][e][cl], sbytes) + lconst;
        const TI *pr = reinterpret_cast<const TI *>(in_re + off), *pi = reinterpret_cast<const TI *>(in_im + off);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            xr[s] = (TM)pr[s];
            xi[s] = (TM)pi[s];
        }
    };
    auto body = [&](int e, int o, TM(&xr)[S], TM(&xi)[S], TM(&nr)[S], TM(&ni)[S]) {
        const unsigned char *tb = s_tab + o * OSTR;
        load(e + 1, nr, ni);  // the zero block after the last offset
        __builtin_amdgcn_sched_barrier(0);  // issued before this offset's work
        {
            // A_0 log(-t) into row 0 (lane group 0; the others read zeros)
            const double2 lg = *reinterpret_cast<const double2 *>(tb + PQ * ROWB + lout);
            const double x0r = (double)xr[0], x0i = (double)xi[0];
            br[0][0] = fma(x0r, lg.x, fma(-x0i, lg.y, br[0][0]));
            bi[0][0] = fma(x0r, lg.y, fma(x0i, lg.x, bi[0][0]));
            a0r += x0r;
            a0i += x0i;
        }
        typename M::acc_t zr[RB], zi[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            zr[r] = M::zero();
            zi[r] = M::zero();
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            // input scaling y_k = (-t)^-k A_k
            const TM wr = *reinterpret_cast<const TM *>(tb + lin + s * ROWB);
            const TM wi = *reinterpret_cast<const TM *>(tb + lin + s * ROWB + sizeof(TM));
            const TM yr = xr[s] * wr - xi[s] * wi;
            const TM yi = xr[s] * wi + xi[s] * wr;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const TM qv = *reinterpret_cast<const TM *>(reinterpret_cast<const unsigned char *>(s_q) + qaddr +
                                                             (s * RB + r) * 64 * sizeof(TM));
                zr[r] = M::op(qv, yr, zr[r]);
                zi[r] = M::op(qv, yi, zi[r]);
            }
        }
        // the fragments are read from LDS per offset: kept in registers
        // across offsets they would crowd out the second column buffer
        asm volatile("" : "+v"(qaddr));
        // output scaling (-t)^-l (the sign (-1)^l is in Q), accumulated
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const unsigned rb = (unsigned)((r * 16 + M::row(i, g)) * ROWB);
                const double vr = (double)*reinterpret_cast<const TM *>(tb + rb);
                const double vi = (double)*reinterpret_cast<const TM *>(tb + rb + sizeof(TM));
                const double zre = (double)zr[r][i], zim = (double)zi[r][i];
                br[r][i] = fma(-zim, vi, fma(zre, vr, br[r][i]));
                bi[r][i] = fma(zim, vr, fma(zre, vi, bi[r][i]));
            }
        // nothing of the next offset (whose columns are still loading) moves up
        __builtin_amdgcn_sched_barrier(0);
    };
    TM ar[S], ai[S], cr[S], ci[S];
    load(0, ar, ai);
    int e = 0;
    for (; e + 1 < nt; e += 2) {
        const int o0 = ld_uniform(a.tile_ops, e0 + e), o1 = ld_uniform(a.tile_ops, e0 + e + 1);
        body(e, o0, ar, ai, cr, ci);
        body(e + 1, o1, cr, ci, ar, ai);
    }
    if (e < nt) body(e, ld_uniform(a.tile_ops, e0 + e), ar, ai, cr, ci);
    if (!valid) return;
    if (g == 0) {
        const double ls = a.logside[a.level[box]];
        br[0][M::item_of(0)] += a0r * ls;
        bi[0][M::item_of(0)] += a0i * ls;
    }
    TO *op = out + (int64_t)box * a.box_stride + (int64_t)bt * a.bt_stride;
    const bool add = a.xinit[box] != 0;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int l = r * 16 + M::row(i, g);
            if (l < P) {
                op[l] = (TO)(add ? (double)op[l] + br[r][i] : br[r][i]);
                op[P + l] = (TO)(add ? (double)op[P + l] + bi[r][i] : bi[r][i]);
            }
        }
    for (int row = 2 * P + g; row < a.PD; row += 4) op[row] = (TO)0;
}

}  // namespace vp

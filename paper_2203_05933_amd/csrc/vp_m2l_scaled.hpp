// M2L in diagonally scaled form on matrix cores.
//
// With the side-scaled expansions of this library the M2L operator for a
// source box at (target centre + s t) factors as
//     B_0 = A_0 (log s + log(-t)) + sum_{k>=1} y_k
//     B_l = t^-l [ -A_0 / l + sum_{k>=1} C(l+k-1, k-1) y_k ],   l >= 1
// with y_k = (-t)^-k A_k: a complex diagonal scaling of the source column,
// ONE real matrix Q (Q[0][k] = 1, Q[l][0] = -1/l, Q[l][k] = C(l+k-1, k-1),
// Q[0][0] = 0) that is the same for all 40 offsets, and a complex diagonal
// scaling of the result.  Because Q is real it acts on the real and the
// imaginary parts separately: the contraction per translation is two real
// P x P products instead of one real 2P x 2P product, and no per-offset
// operator is read from memory.  The terms summed are the same products as
// in the unfactored operator (only their grouping differs), so the rounding
// behaviour is that of the plain operator.
//
// Work split: a 16-column tile (boxes x densities, grouped by child class
// so the tile shares its offsets) per workgroup; the four waves take every
// fourth offset present in the tile (listed at plan time) and their partial
// sums are added through LDS in a fixed order.
#pragma once

#include "vp_translate.hpp"

namespace vp {

struct M2LScaledArgs {
    const int32_t *cols_box;  // box of column group c / nbatch
    int ncols;                // (box, density) columns
    int nbatch;
    const int32_t *slots;     // [box][NOFF] source box or -1
    const int32_t *tile_ptr;  // offsets present in 16-column tile t: tile_ops[tile_ptr[t] .. tile_ptr[t+1])
    const int32_t *tile_ops;
    const int32_t *tile_order;  // launch order of the tiles (most offsets first)
    int P;                    // complex coefficients per expansion
    ColAddr in, out;          // expansion columns (PD rows: re 0..P-1, im P..2P-1)
    int PD;
    const int32_t *level;
    const double *logside;    // log of the box side per level
};

// Q in A-fragment order [rb][s][lane]; tin/tout [NOFF][RB*16][2] (re, im);
// logt [NOFF][2] = log(-t).
template <class TI, class TO, class TM, int RB>
__global__ void __launch_bounds__(256) k_m2l_scaled(M2LScaledArgs a, const TM *__restrict__ Qf,
                                                    const TM *__restrict__ tin, const TM *__restrict__ tout,
                                                    const double *__restrict__ logt, const TI *__restrict__ in,
                                                    TO *__restrict__ out) {
    typedef Mfma<TM> M;
    constexpr int S = RB * 4;  // 4-row steps of the input (RB*16 rows)
    constexpr int PQ = RB * 16;
    constexpr int NR = RB * 4 * 2 + 2;  // reduced values per lane: B re/im per item, A_0 sum re/im
    __shared__ double red[3][NR][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int cl = lane & 15, g = lane >> 4;
    const int tile = a.tile_order[blockIdx.x];
    const int col = tile * 16 + cl;
    const bool valid = col < a.ncols;
    const int box = valid ? a.cols_box[col / a.nbatch] : 0;
    const int bt = valid ? col % a.nbatch : 0;
    const int P = a.P;

    TM q[RB][S];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int s = 0; s < S; ++s) q[r][s] = Qf[(r * S + s) * 64 + lane];

    double br[RB][4], bi[RB][4];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) br[r][i] = bi[r][i] = 0.0;
    double a0r = 0.0, a0i = 0.0;  // sum of A_0 over the sources (lanes g == 0)

    // the tile's offsets and each column's source per offset, staged in LDS
    // once (no dependent global loads inside the loop)
    __shared__ int32_t s_ops[NOFF];
    __shared__ int32_t s_src[NOFF][16];
    const int e0 = a.tile_ptr[tile], nt = a.tile_ptr[tile + 1] - e0;
    for (int i = tid; i < nt; i += 256) s_ops[i] = a.tile_ops[e0 + i];
    __syncthreads();
    for (int i = tid; i < nt * 16; i += 256) {
        const int oi = i >> 4, c = i & 15, cc = tile * 16 + c;
        s_src[oi][c] = cc < a.ncols ? a.slots[(int64_t)a.cols_box[cc / a.nbatch] * NOFF + s_ops[oi]] : -1;
    }
    __syncthreads();

    // this wave's offsets: every fourth one present in the tile; the source
    // columns of the next offset are loaded while the current one is on the
    // matrix cores
    const int e1 = nt;
    int e = wave;
    int o = 0, src = -1;
    TM xr[S], xi[S];
    if (e < e1) {
        o = s_ops[e];
        src = s_src[e][cl];
        const TI *ip = in + (src >= 0 ? a.in.off(src) + (int64_t)bt * a.in.bstride : 0);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int k = 4 * s + g;
            const bool ok = src >= 0 && k < P;
            xr[s] = ok ? (TM)ip[k] : (TM)0;
            xi[s] = ok ? (TM)ip[P + k] : (TM)0;
        }
    }
    while (e < e1) {
        const TM *ti = tin + (size_t)o * PQ * 2;
        TM yr[S], yi[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int k = 4 * s + g;
            const TM wr = ti[2 * k], wi = ti[2 * k + 1];
            yr[s] = xr[s] * wr - xi[s] * wi;
            yi[s] = xr[s] * wi + xi[s] * wr;
        }
        if (g == 0 && src >= 0) {
            // A_0 log(-t): the offset-dependent part of the k = 0 column
            const double x0r = (double)xr[0], x0i = (double)xi[0];
            const double lr = logt[2 * o], li = logt[2 * o + 1];
            br[0][M::item_of(0)] += x0r * lr - x0i * li;
            bi[0][M::item_of(0)] += x0r * li + x0i * lr;
            a0r += x0r;
            a0i += x0i;
        }
        // prefetch the next offset's source columns
        const int en = e + 4;
        int on = 0, srcn = -1;
        if (en < e1) {
            on = s_ops[en];
            srcn = s_src[en][cl];
            const TI *ip = in + (srcn >= 0 ? a.in.off(srcn) + (int64_t)bt * a.in.bstride : 0);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int k = 4 * s + g;
                const bool ok = srcn >= 0 && k < P;
                xr[s] = ok ? (TM)ip[k] : (TM)0;
                xi[s] = ok ? (TM)ip[P + k] : (TM)0;
            }
        }
        typename M::acc_t zr[RB], zi[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            zr[r] = M::zero();
            zi[r] = M::zero();
        }
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                zr[r] = M::op(q[r][s], yr[s], zr[r]);
                zi[r] = M::op(q[r][s], yi[s], zi[r]);
            }
        const TM *to = tout + (size_t)o * PQ * 2;
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
        e = en;
        o = on;
        src = srcn;
    }
    // fixed-order sum of the four waves' partial results
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
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int e = (r * 4 + i) * 2;
            br[r][i] = ((br[r][i] + red[0][e][lane]) + red[1][e][lane]) + red[2][e][lane];
            bi[r][i] = ((bi[r][i] + red[0][e + 1][lane]) + red[1][e + 1][lane]) + red[2][e + 1][lane];
        }
    a0r = ((a0r + red[0][NR - 2][lane]) + red[1][NR - 2][lane]) + red[2][NR - 2][lane];
    a0i = ((a0i + red[0][NR - 1][lane]) + red[1][NR - 1][lane]) + red[2][NR - 1][lane];
    if (g == 0) {
        const double ls = a.logside[a.level[box]];
        br[0][M::item_of(0)] += a0r * ls;
        bi[0][M::item_of(0)] += a0i * ls;
    }
    TO *op = out + a.out.off(box) + (int64_t)bt * a.out.bstride;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int l = r * 16 + M::row(i, g);
            if (l < P) {
                op[l] = (TO)br[r][i];
                op[P + l] = (TO)bi[r][i];
            }
        }
    for (int row = 2 * P + g; row < a.PD; row += 4) op[row] = (TO)0;
}

}  // namespace vp

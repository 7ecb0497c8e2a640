// Evaluation kernels of the volume-potential hot path.
//
// One evaluation of u_b(t_i) = sum_j G(r_j, t_i) w_j f_b(r_j) + (C f_b)(t_i)
// (smooth rule of Section 3.2, eq. Tk_smooth_quad; box rule of Section 4.2;
// Green's function of Section 2.1; correction matrix of Section 4) runs as:
//   charge     q_b[j] = w_j f_b[perm[j]]                (sorted source order)
//   P2M        leaf multipoles; congruent leaves by one matrix (MFMA), others
//              and the virtual children of X-list sources on the VALU
//   M2M        upward pass, level by level             (VALU, scaled form)
//   M2L        V lists, one launch for all levels      (MFMA, scaled form)
//   P2L        X lists two or more levels apart        (VALU)
//   L2L        downward pass, level by level           (VALU, scaled form)
//   tables     near field of congruent leaves          (MFMA, FP64)
//   P2P        remaining U-list pairs, LDS-staged      (FP64 VALU)
//   L2P + M2P  local expansion and W lists at targets  (VALU; MFMA for
//              congruent leaves)
//   finish     u = acc[inverse perm] + C f             (HBM bound)
// The adjoint runs the same passes with the point roles swapped (charges
// g at the targets, evaluated at the nodes, times w) plus C^T g.
// Expansions are [box][batch][PD] columns: rows 0..P-1 real parts,
// P..2P-1 imaginary parts, zero padding; float64, or float32 in the
// FP32-bulk form.  Every reduction has a fixed order: no atomics.

#include <algorithm>
#include <map>
#include <unordered_map>

#include "vp_internal.hpp"
#include "vp_translate.hpp"
#include "vp_m2l_scaled.hpp"

namespace vp {

struct Cplx {
    double re, im;
};

template <class E>
struct C2 {
    E re, im;
};

template <class E>
__device__ inline C2<E> cmul(C2<E> a, C2<E> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

__device__ inline double vp_log(double x);  // defined with the near-field kernel

// Point-set view: which points act as sources and which as targets.
struct PointRoles {
    const double *sx, *sy;         // source coordinates (sorted)
    const int32_t *sb, *se;        // per box source range
    const double *tx, *ty;         // target coordinates (sorted)
    const int32_t *tb, *te;        // per box target range
    int64_t nsrc, ntgt;
};

struct BoxGeo {
    const int32_t *level, *ix, *iy, *parent, *child, *nchild;
    const double *cx, *cy, *side, *logside;
};

// ----------------------------------------------------------------------------
// charges
// ----------------------------------------------------------------------------
// q[b][i] = w_i f_b[perm i]
__global__ void k_charge(const double *__restrict__ f, const int32_t *__restrict__ perm,
                         const double *__restrict__ w, double *__restrict__ q, int64_t len, int nbatch) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    int32_t j = perm[i];
    double wi = w ? w[i] : 1.0;
    for (int b = 0; b < nbatch; ++b) q[(int64_t)b * len + i] = wi * f[(int64_t)b * len + j];
}

// The same, and qi[i][b] (density fastest) through an LDS transpose of the
// workgroup's 64 points x nbatch densities, so that both stores write whole
// contiguous rows (q == nullptr: only qi).  Dynamic LDS: 64 (nbatch + 1) doubles.
__global__ void __launch_bounds__(64) k_charge_il(const double *__restrict__ f, const int32_t *__restrict__ perm,
                                                  const double *__restrict__ w, double *__restrict__ q,
                                                  int64_t len, int nbatch, double *__restrict__ qi) {
    extern __shared__ double tile[];  // [point][nbatch + 1]
    const int ld = nbatch + 1;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int li = threadIdx.x;
    const int64_t i = i0 + li;
    if (i < len) {
        const int32_t j = perm[i];
        const double wi = w ? w[i] : 1.0;
        for (int b = 0; b < nbatch; ++b) {
            const double v = wi * f[(int64_t)b * len + j];
            if (q) q[(int64_t)b * len + i] = v;
            tile[li * ld + b] = v;
        }
    }
    __syncthreads();
    const int npts = (int)min<int64_t>(64, len - i0);
    // element e = pi nbatch + b of the block; one division, then steps of 64
    const int dq = 64 / nbatch, dr = 64 - dq * nbatch;
    int pi = li / nbatch, b = li - pi * nbatch;
    double *out = qi + i0 * nbatch;
    for (int e = li; e < npts * nbatch; e += 64) {
        out[e] = tile[pi * ld + b];
        pi += dq;
        b += dr;
        if (b >= nbatch) {
            b -= nbatch;
            ++pi;
        }
    }
}

// Charges and the leaf P2M in one pass, for forward evaluations whose only
// charge readers are the near tables (density-fastest copy) and the P2M of
// pattern leaves, with 16 densities: a wave takes one leaf's 16 densities,
// forms the charges w_k f_d[perm k] of its sorted nodes k = 4 s + g, stores
// them density-fastest and multiplies them by the P2M matrix (A: RB x S
// fragments, the product order of k_fixed_apply, so the multipoles are the
// same to the bit; TM float: the FP32-bulk form, charges rounded to FP32 for
// the product as there).  Multipoles of box b, density d, row r at
// Mx[b * 16 PD + d PD + r].
template <class TM, int RB, int S>
__global__ void __launch_bounds__(256) k_p2m_charge(const int32_t *__restrict__ leaves, int nleaf,
                                                    const int32_t *__restrict__ sb, const int32_t *__restrict__ perm,
                                                    const double *__restrict__ w, const double *__restrict__ f,
                                                    int64_t flen, const TM *__restrict__ A,
                                                    double *__restrict__ qi, TM *__restrict__ Mx, int PD) {
    typedef Mfma<TM> M;
    constexpr int AE = RB * S * 64;
    __shared__ TM sA[AE];
    for (int e = threadIdx.x; e < AE; e += blockDim.x) sA[e] = A[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, cl = lane & 15, g = lane >> 4;
    const int stride = (int)gridDim.x * 4;
    int j = (int)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (j >= nleaf) return;
    const double *fd = f + (int64_t)cl * flen;
    // sorted node indices and weights of leaf jj (element k = 4 s + g)
    auto first = [&](int jj) { return ld_uniform(sb, ld_uniform(leaves, jj)) + g; };
    auto ld_perm = [&](int jj, int (&ix)[S]) {
        const int s0 = first(jj);
#pragma unroll
        for (int s = 0; s < S; ++s) ix[s] = perm[s0 + 4 * s];
    };
    auto ld_w = [&](int jj, double (&wv)[S]) {
        const int s0 = first(jj);
#pragma unroll
        for (int s = 0; s < S; ++s) wv[s] = w[s0 + 4 * s];
    };
    auto next = [&](int jj) { return jj + stride < nleaf ? jj + stride : jj; };
    // pipeline: this leaf's charges x and the next leaf's node indices and
    // weights; per leaf the next leaf's density values are requested, then
    // the indices of the one after, before this leaf's products, and the
    // weights of the one after once the next leaf's charges are formed
    int ix[S];
    double wv[S], x[S];
    ld_perm(j, ix);
    ld_w(j, wv);
#pragma unroll
    for (int s = 0; s < S; ++s) x[s] = wv[s] * fd[ix[s]];
    int jn = next(j);
    ld_perm(jn, ix);
    ld_w(jn, wv);
    for (; j < nleaf; j += stride) {
        const int box = ld_uniform(leaves, j);
        const int s0 = ld_uniform(sb, box);
        double *qo = qi + ((int64_t)s0 + g) * 16 + cl;
#pragma unroll
        for (int s = 0; s < S; ++s) qo[64 * s] = x[s];
        double fv[S];
#pragma unroll
        for (int s = 0; s < S; ++s) fv[s] = fd[ix[s]];
        const int jn2 = next(jn);
        ld_perm(jn2, ix);
        typename M::acc_t acc[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[r] = M::zero();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            TM a_s[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) a_s[r] = sA[(r * S + s) * 64 + lane];
#pragma unroll
            for (int r = 0; r < RB; ++r) acc[r] = M::op((TM)x[s], a_s[r], acc[r]);
            __builtin_amdgcn_sched_barrier(0);
        }
        TM *mo = Mx + (int64_t)box * 16 * PD + cl;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int r = 0; r < RB; ++r) mo[M::row(i, g) * PD + r * 16] = acc[r][i];
#pragma unroll
        for (int s = 0; s < S; ++s) x[s] = wv[s] * fv[s];
        ld_w(jn2, wv);
        jn = jn2;
    }
}

// ----------------------------------------------------------------------------
// Power tables for P2M / P2L.  Sources come in chunks of 16; lane
// (j = l % 16, g = l / 16) fills entries k in [g*KP, (g+1)*KP) of row j,
// starting from w^(g*KP) obtained by repeated squaring, so all 64 lanes
// work.  Row j holds c_k w_j^k (c_0 = the k = 0 entry, c_k = -1/k).
// ----------------------------------------------------------------------------
template <class E>
__device__ inline C2<E> cpow_int(C2<E> w, int n) {
    C2<E> r = {(E)1, (E)0};
    while (n > 0) {
        if (n & 1) r = cmul(r, w);
        w = cmul(w, w);
        n >>= 1;
    }
    return r;
}

template <class E>
__device__ inline void fill_power_rows(C2<E> w, E k0re, bool valid, int j, int g, int P, E *Wre, E *Wim) {
    const int KP = (P + 3) / 4;
    const int k0 = g * KP, k1 = min(P, k0 + KP);
    if (!valid) {
        for (int k = k0; k < k1; ++k) {
            Wre[j * P + k] = (E)0;
            Wim[j * P + k] = (E)0;
        }
        return;
    }
    C2<E> pw = cpow_int(w, k0);
    for (int k = k0; k < k1; ++k) {
        if (k == 0) {
            Wre[j * P] = k0re;
            Wim[j * P] = (E)0;
        } else {
            Wre[j * P + k] = pw.re;  // the factor -1/k is applied to the sums
            Wim[j * P + k] = pw.im;
        }
        pw = cmul(pw, w);
    }
}

// ----------------------------------------------------------------------------
// P2M: one wave per leaf; A_k = -(1/k) sum_j q_j W[j][k] in source order
// (A_0 = sum_j q_j), with W[j][k] = ((z_j - c)/s)^k.
// ----------------------------------------------------------------------------
template <class E>
__device__ inline void p2m_range(const PointRoles &R, int s0, int s1, double cx, double cy, double inv_s,
                                 const double *__restrict__ q, int nbatch, int P, int PD,
                                 const E *__restrict__ invk, E *__restrict__ out, E *Wre, E *Wim,
                                 E (*sq)[16]) {
    const int lane = threadIdx.x, j = lane & 15, g = lane >> 4;
    for (int bt0 = 0; bt0 < nbatch; bt0 += 16) {
        const int nbg = min(16, nbatch - bt0);
        E acc[2][16];
        for (int k = 0; k < 16; ++k) acc[0][k] = acc[1][k] = (E)0;
        for (int base = s0; base < s1; base += 16) {
            const int cnt = min(16, s1 - base);
            __syncthreads();
            const bool v = j < cnt;
            const int jj = base + (v ? j : 0);
            const C2<E> w = {(E)((R.sx[jj] - cx) * inv_s), (E)((R.sy[jj] - cy) * inv_s)};
            fill_power_rows<E>(w, (E)1, v, j, g, P, Wre, Wim);
            for (int bb = g; bb < nbg; bb += 4) sq[bb][j] = v ? (E)q[(int64_t)(bt0 + bb) * R.nsrc + jj] : (E)0;
            __syncthreads();
            // static register indexing (rows r = lane + 64 ri, densities bb)
#pragma unroll
            for (int ri = 0; ri < 2; ++ri) {
                const int r = lane + 64 * ri;
                if (r < 2 * P) {
                    const int k = r < P ? r : r - P;
                    const E *Wc = r < P ? Wre : Wim;
#pragma unroll
                    for (int bb = 0; bb < 16; ++bb) {
                        if (bb < nbg) {
                            E t = (E)0;
                            for (int jx = 0; jx < cnt; ++jx) t += sq[bb][jx] * Wc[jx * P + k];
                            acc[ri][bb] += t;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) {
            const int r = lane + 64 * ri;
            if (r < PD) {
                const int k = r < P ? r : r - P;
                const E sc = r >= 2 * P ? (E)0 : (k == 0 ? (E)1 : -invk[k]);
#pragma unroll
                for (int bb = 0; bb < 16; ++bb)
                    if (bb < nbg) out[(bt0 + bb) * PD + r] = sc * acc[ri][bb];
            }
        }
    }
}

// VALU P2M, one wave per job (a leaf about its centre at its scale, or the
// quadrant of an X-list source leaf about the quadrant centre at the
// children's scale), from a plan-time descriptor.
template <class E>
__global__ void __launch_bounds__(64) k_p2m(PointRoles R, const P2MJob *__restrict__ jobs,
                                            const double *__restrict__ q, int nbatch, int P, int PD,
                                            const E *__restrict__ invk, E *__restrict__ Mexp) {
    extern __shared__ unsigned char smem[];
    E *Wre = reinterpret_cast<E *>(smem);   // [16][P]
    E *Wim = Wre + 16 * P;                  // [16][P]
    __shared__ E sq[16][16];                // charges of the chunk [density][source]
    const P2MJob jb = jobs[blockIdx.x];
    p2m_range<E>(R, jb.s0, jb.s1, jb.cx, jb.cy, jb.inv_s, q, nbatch, P, PD, invk,
                 Mexp + (int64_t)jb.col * nbatch * PD, Wre, Wim, sq);
}

// ----------------------------------------------------------------------------
// M2M on the VALU in diagonally scaled form: one wave per parent box of a
// level.  Every child column is scaled by tin[class][k], multiplied by the
// real matrix Q (shared by all classes; read transposed so a wave's loads are
// contiguous), scaled by tout[class][l] and summed.  A lane owns output row l
// of one group of quadrants; with P <= 32 the wave's halves (quarters for
// P <= 16) take alternate quadrants and are added through LDS in a fixed
// order.  The children come from a plan-time table [parent][quadrant] (the
// quadrant is the child's class), so the child columns load one round trip
// after the launch-list entry.
// ----------------------------------------------------------------------------
template <class E, int PR>
__global__ void __launch_bounds__(64) k_m2m(const int32_t *__restrict__ boxes, const int4 *__restrict__ cslot,
                                            int nbatch, int P, int PD, const E *__restrict__ QT,
                                            const E *__restrict__ tin, const E *__restrict__ tout,
                                            E *__restrict__ X, int chunk) {
    constexpr int H = 64 / PR;       // row groups in the wave
    __shared__ E ys[4][PR][2];       // scaled child columns (re, im interleaved)
    __shared__ E red[H][PR][2];      // per-group partial rows
    const int lane = threadIdx.x;
    const int gi = lane / PR, l = lane % PR;
    E qc[PR];  // this lane's row of Q (column l of QT), kept in registers
#pragma unroll
    for (int k = 0; k < PR; ++k) qc[k] = (k < P && l < P) ? QT[k * PR + l] : (E)0;
    const int b = boxes[blockIdx.x];
    const int4 cs = cslot[blockIdx.x];
    auto child = [&](int c) { return c == 0 ? cs.x : (c == 1 ? cs.y : (c == 2 ? cs.z : cs.w)); };
    const int bt_end = min(nbatch, (int)(blockIdx.y + 1) * chunk);
    for (int bt = blockIdx.y * chunk; bt < bt_end; ++bt) {
#pragma unroll
        for (int j = 0; j < 4 / H; ++j) {
            const int c = gi + H * j, ch = child(c);
            E yr = (E)0, yi = (E)0;
            if (l < P && ch >= 0) {
                const E *x = X + ((int64_t)ch * nbatch + bt) * PD;
                const E xr = x[l], xi = x[P + l];
                const E wr = tin[(c * P + l) * 2], wi = tin[(c * P + l) * 2 + 1];
                yr = xr * wr - xi * wi;
                yi = xr * wi + xi * wr;
            }
            ys[c][l][0] = yr;
            ys[c][l][1] = yi;
        }
        __syncthreads();
        E br = (E)0, bi = (E)0;
#pragma unroll
        for (int j = 0; j < 4 / H; ++j) {
            const int c = gi + H * j;
            if (child(c) < 0) continue;
            E zr = (E)0, zi = (E)0;
#pragma unroll
            for (int k = 0; k < PR; ++k) {
                zr += qc[k] * ys[c][k][0];
                zi += qc[k] * ys[c][k][1];
            }
            if (l < P) {
                const E vr = tout[(c * P + l) * 2], vi = tout[(c * P + l) * 2 + 1];
                br += zr * vr - zi * vi;
                bi += zr * vi + zi * vr;
            }
        }
        if (H > 1) {
            red[gi][l][0] = br;
            red[gi][l][1] = bi;
            __syncthreads();
            if (gi == 0) {
#pragma unroll
                for (int h = 1; h < H; ++h) {
                    br += red[h][l][0];
                    bi += red[h][l][1];
                }
            }
        }
        E *o = X + ((int64_t)b * nbatch + bt) * PD;
        if (gi == 0 && l < P) {
            o[l] = br;
            o[P + l] = bi;
        }
        for (int r = 2 * P + lane; r < PD; r += 64) o[r] = (E)0;
        __syncthreads();
    }
}

// The same M2M on the matrix cores when a 16-column tile is one parent's
// sixteen densities (nbatch a multiple of 16, FP64): one tile per wave, the
// children's columns scaled on the VALU, multiplied by Q as in k_m2l_wave
// (Q's fragments and the scaling tables in LDS, Q staged from its transposed
// copy) and the scaled results summed over the four children.  A child's
// columns load while the previous child's products run; an absent child
// reads the multipole array's zero block (zero_box).
template <int RB>
__global__ void __launch_bounds__(256) k_m2m_wave(const int32_t *__restrict__ parents,
                                                  const int4 *__restrict__ cslot, int nparents, int nbatch, int P,
                                                  int PD, int PR, int zero_box, const double *__restrict__ QT,
                                                  const double *__restrict__ tin, const double *__restrict__ tout,
                                                  double *__restrict__ X) {
    typedef Mfma<double> M;
    constexpr int S = RB * 4, PQ = RB * 16;
    __shared__ __align__(16) double s_q[RB * S * 64];  // [s][r][lane]
    __shared__ __align__(16) double s_in[4][PQ][2], s_out[4][PQ][2];
    const int tid = threadIdx.x, lane = tid & 63, cl = lane & 15, g = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int i = tid; i < RB * S * 64; i += 256) {
        const int st = i / (RB * 64), r = (i / 64) % RB, l = i & 63;
        const int k = (l >> 4) * S + st, row = r * 16 + (l & 15);
        s_q[i] = k < P && row < P ? QT[k * PR + row] : 0.0;
    }
    for (int i = tid; i < 4 * PQ; i += 256) {
        const int c = i / PQ, k = i % PQ;
        const bool in = k < P;
        s_in[c][k][0] = in ? tin[(c * P + k) * 2] : 0.0;
        s_in[c][k][1] = in ? tin[(c * P + k) * 2 + 1] : 0.0;
        s_out[c][k][0] = in ? tout[(c * P + k) * 2] : 0.0;
        s_out[c][k][1] = in ? tout[(c * P + k) * 2 + 1] : 0.0;
    }
    __syncthreads();
    const int tpp = nbatch / 16;  // tiles per parent
    const int t = blockIdx.x * 4 + wave;
    if (t >= nparents * tpp) return;
    const int pi = t / tpp, d0 = (t - pi * tpp) * 16;
    const int pb = ld_uniform(parents, pi);
    const int32_t *cs = reinterpret_cast<const int32_t *>(cslot) + 4 * pi;
    const int64_t lane_off = (int64_t)(d0 + cl) * PD + g * S;
    // an absent child reads the zero block
    auto load = [&](int c, double(&xr)[S], double(&xi)[S]) {
        const int chc = ld_uniform(cs, c);
        const double *x = X + (int64_t)(chc >= 0 ? chc : zero_box) * nbatch * PD + lane_off;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            xr[s] = x[s];
            xi[s] = x[P + s];
        }
    };
    double br[RB][4], bi[RB][4];
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) br[r][i] = bi[r][i] = 0.0;
    unsigned qaddr = (unsigned)lane * 8u;
    auto child = [&](int c, const double(&xr)[S], const double(&xi)[S]) {
        typename M::acc_t zr[RB], zi[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) zr[r] = zi[r] = M::zero();
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int k = g * S + s;
            const double wr = s_in[c][k][0], wi = s_in[c][k][1];
            const double yr = xr[s] * wr - xi[s] * wi, yi = xr[s] * wi + xi[s] * wr;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const double q = *reinterpret_cast<const double *>(reinterpret_cast<const char *>(s_q) + qaddr +
                                                                   (s * RB + r) * 64 * 8);
                zr[r] = M::op(q, yr, zr[r]);
                zi[r] = M::op(q, yi, zi[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int l = r * 16 + M::row(i, g);
                const double vr = s_out[c][l][0], vi = s_out[c][l][1];
                br[r][i] = fma(-zi[r][i], vi, fma(zr[r][i], vr, br[r][i]));
                bi[r][i] = fma(zi[r][i], vr, fma(zr[r][i], vi, bi[r][i]));
            }
    };
    // each child's columns load during the previous child's products; Q's
    // fragments are read from LDS per child (kept in registers across the
    // children they would cost a wave per SIMD)
    double ar[S], ai[S], nr[S], ni[S];
    load(0, ar, ai);
#pragma unroll 1
    for (int c = 0; c < 4; ++c) {
        load(c < 3 ? c + 1 : 3, nr, ni);  // (the last child again after the last: loaded, unused)
        child(c, ar, ai);
        asm volatile("" : "+v"(qaddr));
#pragma unroll
        for (int s = 0; s < S; ++s) {
            ar[s] = nr[s];
            ai[s] = ni[s];
        }
    }
    double *o = X + ((int64_t)pb * nbatch + d0 + cl) * PD;
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int l = r * 16 + M::row(i, g);
            if (l < P) {
                o[l] = br[r][i];
                o[P + l] = bi[r][i];
            }
        }
    for (int row = 2 * P + g; row < PD; row += 4) o[row] = 0.0;
}

// L2L in the same scaled form (Q upper triangular), one target box per row
// group: a wave serves 64 / PR boxes of a level, each row group staging its
// own parent column.  The launch list carries parent * 4 + class beside each
// box, so the parent column, the box's own column and the scalings all load
// one round trip after the list entry.
template <class E, int PR>
__global__ void __launch_bounds__(64) k_l2l(const int32_t *__restrict__ boxes, const int32_t *__restrict__ pcls,
                                            int nboxes, int nbatch, int P, int PD, const E *__restrict__ QT,
                                            const E *__restrict__ tin, const E *__restrict__ tout,
                                            E *__restrict__ X, int chunk) {
    constexpr int H = 64 / PR;
    __shared__ E ys[H][PR][2];
    const int lane = threadIdx.x;
    const int gi = lane / PR, l = lane % PR;
    E qc[PR];
#pragma unroll
    for (int k = 0; k < PR; ++k) qc[k] = (k < P && l < P) ? QT[k * PR + l] : (E)0;
    const int idx = blockIdx.x * H + gi;
    const bool act = idx < nboxes;
    const int b = act ? boxes[idx] : 0;
    const int pc = act ? pcls[idx] : 0;
    const int src = pc >> 2, cls = pc & 3;
    const bool row = act && l < P;
    E wr = (E)0, wi = (E)0, vr = (E)0, vi = (E)0;
    if (row) {
        wr = tin[(cls * P + l) * 2];
        wi = tin[(cls * P + l) * 2 + 1];
        vr = tout[(cls * P + l) * 2];
        vi = tout[(cls * P + l) * 2 + 1];
    }
    const int bt_end = min(nbatch, (int)(blockIdx.y + 1) * chunk);
    for (int bt = blockIdx.y * chunk; bt < bt_end; ++bt) {
        E yr = (E)0, yi = (E)0, or_ = (E)0, oi = (E)0;
        E *o = X + ((int64_t)b * nbatch + bt) * PD;
        if (row) {
            const E *x = X + ((int64_t)src * nbatch + bt) * PD;
            const E xr = x[l], xi = x[P + l];
            or_ = o[l];
            oi = o[P + l];
            yr = xr * wr - xi * wi;
            yi = xr * wi + xi * wr;
        }
        ys[gi][l][0] = yr;
        ys[gi][l][1] = yi;
        __syncthreads();
        E zr = (E)0, zi = (E)0;
#pragma unroll
        for (int k = 0; k < PR; ++k) {
            zr += qc[k] * ys[gi][k][0];
            zi += qc[k] * ys[gi][k][1];
        }
        if (row) {
            o[l] = or_ + (zr * vr - zi * vi);
            o[P + l] = oi + (zr * vi + zi * vr);
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------
// P2L (X lists): sources of coarser leaves straight into the local expansion
// of box b: B_0 = sum q log|c - z|, B_l = -(1/l) sum q (s/(z - c))^l over all
// of b's entries.  It writes the column; M2L then adds its translations.
// ----------------------------------------------------------------------------
template <class E>
__global__ void __launch_bounds__(64) k_p2l(PointRoles R, BoxGeo G, const int32_t *__restrict__ boxes,
                                            const int32_t *__restrict__ xptr,
                                            const int32_t *__restrict__ xidx,
                                            const double *__restrict__ q, int nbatch, int P, int PD,
                                            const E *__restrict__ invk, E *__restrict__ Lexp) {
    extern __shared__ unsigned char smem[];
    E *Wre = reinterpret_cast<E *>(smem);  // [16][P]
    E *Wim = Wre + 16 * P;
    __shared__ E sq[16][16];               // charges of the chunk [density][source]
    const int lane = threadIdx.x, j = lane & 15, g = lane >> 4;
    const int b = boxes[blockIdx.x];
    const double cx = G.cx[b], cy = G.cy[b];
    const double s = G.side[G.level[b]];
    E *Lo = Lexp + (int64_t)b * nbatch * PD;
    for (int bt0 = 0; bt0 < nbatch; bt0 += 16) {
        const int nb = min(16, nbatch - bt0);
        E acc[2][16];
        for (int k = 0; k < 16; ++k) acc[0][k] = acc[1][k] = (E)0;
        for (int e = xptr[b]; e < xptr[b + 1]; ++e) {
            const int a = xidx[e];
            const int s0 = R.sb[a], s1 = R.se[a];
            for (int base = s0; base < s1; base += 16) {
                const int cnt = min(16, s1 - base);
                __syncthreads();
                const bool v = j < cnt;
                const int jj = base + (v ? j : 0);
                const double dx = R.sx[jj] - cx, dy = R.sy[jj] - cy;
                const double d2 = dx * dx + dy * dy;
                // s / (z - c) = s (dx - i dy) / d2
                const C2<E> iw = {(E)(s * dx / d2), (E)(-s * dy / d2)};
                fill_power_rows<E>(iw, (E)(0.5 * vp_log(d2)), v, j, g, P, Wre, Wim);
                for (int bb = g; bb < nb; bb += 4) sq[bb][j] = v ? (E)q[(int64_t)(bt0 + bb) * R.nsrc + jj] : (E)0;
                __syncthreads();
#pragma unroll
                for (int ri = 0; ri < 2; ++ri) {
                    const int r = lane + 64 * ri;
                    if (r < 2 * P) {
                        const int k = r < P ? r : r - P;
                        const E *Wc = r < P ? Wre : Wim;
#pragma unroll
                        for (int bb = 0; bb < 16; ++bb) {
                            if (bb < nb) {
                                E t = (E)0;
                                for (int jx = 0; jx < cnt; ++jx) t += sq[bb][jx] * Wc[jx * P + k];
                                acc[ri][bb] += t;
                            }
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int ri = 0; ri < 2; ++ri) {
            const int r = lane + 64 * ri;
            if (r < 2 * P) {
                const int k = r < P ? r : r - P;
                const E sc = k == 0 ? (E)1 : -invk[k];
#pragma unroll
                for (int bb = 0; bb < 16; ++bb)
                    if (bb < nb) Lo[(bt0 + bb) * PD + r] = sc * acc[ri][bb];
            }
        }
    }
}

// ----------------------------------------------------------------------------
// L2P and/or M2P at the targets of one leaf (one wave, lane = target):
//   u += -(1/2pi) Re[ sum_l B_l w^l + sum_{a in W} (A_0 log(z - c_a) +
//                    sum_k A_k (s_a/(z - c_a))^k) ]
// and, with grad, the gradient -(1/2pi) (Re phi', -Im phi').
// ----------------------------------------------------------------------------
template <class E, bool GRAD>
__global__ void __launch_bounds__(256) k_far(PointRoles R, BoxGeo G, const int32_t *__restrict__ leaves,
                                             const int32_t *__restrict__ wptr,
                                             const int32_t *__restrict__ widx, int nbatch, int P,
                                             int PD, const E *__restrict__ Mexp,
                                             const E *__restrict__ Lexp,
                                             const int32_t *__restrict__ local_done,
                                             double *__restrict__ acc, int parts) {
    // Up to four waves per leaf, all on the same 64 targets: wave 0 evaluates
    // the local expansion, wave w takes every nw-th W-list multipole from the
    // w-th on (long W lists of large leaves no longer run on one wave), and
    // the partial sums are added through LDS in a fixed order.  Each wave
    // stages its current coefficient column in its own LDS row (a wave-local
    // barrier suffices, so waves with different list lengths never wait on
    // one another inside the loop).
    constexpr int NR = GRAD ? 2 : 1;
    __shared__ E colw[4][128];
    __shared__ double red[3][NR][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    E *col = colw[wave];
    const int b = leaves[blockIdx.x];
    const int t0 = R.tb[b], t1 = R.te[b];
    if (t1 <= t0) return;
    const double cx = G.cx[b], cy = G.cy[b];
    const int lb = G.level[b];
    const double s = G.side[lb];
    // parts: bit 0 the local expansion, bit 1 the W list
    const bool has_local = (parts & 1) && wave == 0 && lb >= 2 && !(local_done && local_done[b]);
    const int w0 = wptr[b], w1 = (parts & 2) ? wptr[b + 1] : w0;
    for (int base = t0; base < t1; base += 64) {
        const int t = base + lane;
        const bool act = t < t1;
        const double px = act ? R.tx[t] : cx, py = act ? R.ty[t] : cy;
        const C2<E> w = {(E)((px - cx) / s), (E)((py - cy) / s)};
        for (int bt = 0; bt < nbatch; ++bt) {
            C2<E> phi = {(E)0, (E)0}, dphi = {(E)0, (E)0};
            if (has_local) {
                for (int k = lane; k < 2 * P; k += 64) col[k] = Lexp[((int64_t)b * nbatch + bt) * PD + k];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 4
                for (int l = P - 1; l >= 0; --l) {
                    const E cre = col[l], cim = col[P + l];
                    if (GRAD && l >= 1) {
                        dphi = cmul(dphi, w);
                        dphi.re += (E)l * cre;
                        dphi.im += (E)l * cim;
                    }
                    phi = cmul(phi, w);
                    phi.re += cre;
                    phi.im += cim;
                }
                if (GRAD) {
                    dphi.re /= (E)s;
                    dphi.im /= (E)s;
                }
                __builtin_amdgcn_wave_barrier();
            }
            double u = (double)phi.re;
            double gx = (double)dphi.re, gy = -(double)dphi.im;
            for (int e = w0 + wave; e < w1; e += nw) {
                const int a = widx[e];
                for (int k = lane; k < 2 * P; k += 64) col[k] = Mexp[((int64_t)a * nbatch + bt) * PD + k];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const double ax = G.cx[a], ay = G.cy[a], sa = G.side[G.level[a]];
                const double dx = px - ax, dy = py - ay, d2 = dx * dx + dy * dy;
                // iw = s_a / (z - c_a)
                const C2<E> iw = {(E)(sa * dx / d2), (E)(-sa * dy / d2)};
                C2<E> ser = {(E)0, (E)0}, dser = {(E)0, (E)0};
#pragma unroll 4
                for (int k = P - 1; k >= 1; --k) {
                    const E cre = col[k], cim = col[P + k];
                    ser = cmul(ser, iw);
                    ser.re += cre;
                    ser.im += cim;
                    if (GRAD) {
                        dser = cmul(dser, iw);
                        dser.re += (E)k * cre;
                        dser.im += (E)k * cim;
                    }
                }
                ser = cmul(ser, iw);
                const double a0 = (double)col[0];
                __builtin_amdgcn_wave_barrier();  // all lanes done reading col before the next entry's writes
                u += (double)ser.re + a0 * 0.5 * vp_log(d2);
                if (GRAD) {
                    // phi' = (A_0 - sum_k k A_k iw^k) / (z - c)
                    dser = cmul(dser, iw);
                    double nre = a0 - (double)dser.re, nim = -(double)dser.im;
                    // 1/(z - c) = (dx - i dy)/d2
                    double ire = dx / d2, iim = -dy / d2;
                    gx += nre * ire - nim * iim;
                    gy -= nre * iim + nim * ire;
                }
            }
            // fixed-order sum of the waves' partial results (one-wave blocks,
            // used for local expansions alone, skip it)
            if (nw > 1) {
                __syncthreads();
                if (wave > 0) {
                    if (GRAD) {
                        red[wave - 1][0][lane] = gx;
                        red[wave - 1][1][lane] = gy;
                    } else {
                        red[wave - 1][0][lane] = u;
                    }
                }
                __syncthreads();
            }
            if (wave == 0 && act) {
                for (int w2 = 1; w2 < nw; ++w2) {
                    if (GRAD) {
                        gx += red[w2 - 1][0][lane];
                        gy += red[w2 - 1][NR - 1][lane];
                    } else {
                        u += red[w2 - 1][0][lane];
                    }
                }
                if (GRAD) {
                    acc[((int64_t)bt * 2 + 0) * R.ntgt + t] += -INV_2PI * gx;
                    acc[((int64_t)bt * 2 + 1) * R.ntgt + t] += -INV_2PI * gy;
                } else {
                    acc[(int64_t)bt * R.ntgt + t] += -INV_2PI * u;
                }
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Natural logarithm of a positive normal double, for the near field.
// Range reduction x = m 2^e with m in [1/sqrt2, sqrt2), then
//   log m = 2 atanh(s),  s = (m - 1)/(m + 1),  |s| <= 0.1716,
// with the Taylor series atanh(s) = s + s^3/3 + s^5/5 + ... truncated after
// the s^23 term (remainder < 1e-17 relative).  1/(m+1) comes from the
// hardware reciprocal refined by two Newton steps; e log 2 is added with a
// two-part log 2.  Accuracy is a few ulps, far below the 1e-12 target.
// ----------------------------------------------------------------------------
// Series coefficients 2/(2k+3), k = 0..10, in constant memory: uniform
// loads keep them in scalar registers, so each Horner step is one untied FMA.
__constant__ double c_log_series[11] = {2.0 / 3.0,  2.0 / 5.0,  2.0 / 7.0,  2.0 / 9.0,
                                        2.0 / 11.0, 2.0 / 13.0, 2.0 / 15.0, 2.0 / 17.0,
                                        2.0 / 19.0, 2.0 / 21.0, 2.0 / 23.0};

__device__ inline double vp_log(double x) {
    const double SQRT_HALF = 0.70710678118654752440;
    const double LN2_HI = 6.93147180369123816490e-01;  // 0x3FE62E42FEE00000
    const double LN2_LO = 1.90821492927058770002e-10;  // log 2 - LN2_HI
    int e = __builtin_amdgcn_frexp_exp(x);
    double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
    const bool lo = m < SQRT_HALF;
    m = lo ? m + m : m;
    e = lo ? e - 1 : e;
    const double f = m - 1.0;  // exact
    const double d = m + 1.0;
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    const double sv = f * r;
    const double z = sv * sv;
    double pl = c_log_series[10];
#pragma unroll
    for (int k = 9; k >= 0; --k) pl = fma(pl, z, c_log_series[k]);
    const double logm = fma(sv * z, pl, 2.0 * sv);
    const double de = (double)e;
    return fma(de, LN2_HI, fma(de, LN2_LO, logm));
}

// Table-driven base-2 logarithm for the pairwise near field (the
// table-lookup scheme of P. T. P. Tang, ACM TOMS 16, 1990, with our own
// table and series): x = 2^e m, m in [1/2, 1); the top LOG_BITS fraction
// bits i of m select inv_c = fl(1/c_i), c_i the centre of m's interval of
// width 2^-(LOG_BITS+1), and L_i = -log2(inv_c) (both from the host,
// LOG_TABLE entries); u = m inv_c - 1 (one rounding, |u| <= 2^-(LOG_BITS+1))
// and log2 x = e + L_i + u p(u), with p(u) = log2(1 + u)/u by its Taylor
// series through u^LOG_DEG (truncation of u p(u) below 2^-56).  The pair loop
// sums base-2 logarithms and each target's sum is multiplied by log 2 once,
// so the exponent enters as one add instead of a two-part product.
//
// Table layout in LDS: the entry of fraction bits i sits at LOG_BASE + i,
// found from the LOG_BITS fraction bits and the two lowest exponent bits of
// m's high word (10 for every m in [1/2, 1): LOG_BASE = 2^(LOG_BITS+1)).
// x = 0 has m = 0 and e = 0 and so selects entry 0, which holds (0, p(-1)):
// u = -1 and the sum -p(-1) + p(-1) is exactly zero.  A zero distance (the
// self pair) thus contributes exactly nothing without a compare or select in
// the pair loop.  Entries 1 .. LOG_BASE-1 are never read; the kernel keeps
// its source tiles there when they fit.
constexpr int LOG_BASE = 2 << LOG_BITS;
constexpr int LOG_DEG = (56 + LOG_BITS) / (LOG_BITS + 1) - 2;  // smallest D with 2^-(B+1)(D+2) <= 2^-56

__device__ inline double log2p1_over_u(double u) {
    constexpr double IL2 = 1.44269504088896340736;  // 1 / log 2
    // IL2 sum_{k <= LOG_DEG} (-u)^k / (k + 1), by Horner
    double p = ((LOG_DEG & 1) ? -IL2 : IL2) / (LOG_DEG + 1);
#pragma unroll
    for (int k = LOG_DEG - 1; k >= 0; --k) p = fma(u, p, ((k & 1) ? -IL2 : IL2) / (k + 1));
    return p;
}

__device__ inline double vp_log2_tab(double x, const double2 *__restrict__ tab) {
    const int e = __builtin_amdgcn_frexp_exp(x);
    const double m = __builtin_amdgcn_frexp_mant(x);
    const unsigned i = ((unsigned)__double2hiint(m) >> (20 - LOG_BITS)) & ((4u << LOG_BITS) - 1u);
    const double2 t = tab[i];
    const double u = fma(m, t.x, -1.0);
    return (double)e + fma(u, log2p1_over_u(u), t.y);
}

// ----------------------------------------------------------------------------
// P2P (U lists), FP64: one wave per target leaf.  All source points of the
// leaf's list are staged in LDS (SoA x, y, q per density) in tiles of
// P2PCap points, so a leaf with many small neighbours pays one barrier
// pair per tile.  When a leaf has few targets the lanes also split the
// source loop (K lane groups) and the partial sums are combined in a fixed
// order.  Pairs at zero distance (the self pair) contribute nothing: the
// logarithm returns exactly zero there (the table's zero entry), and the
// gradient multiplies its reciprocal by zero, so the loop has no branch.
// ----------------------------------------------------------------------------
template <int NB>
struct P2PCap {
    // small tiles keep a one-wave block's LDS at a few KB, so many waves share a CU
    static constexpr int value = NB <= 2 ? 128 : (NB <= 4 ? 96 : (NB <= 8 ? 64 : 48));
};

template <int NB, bool GRAD, bool ACCUM, bool GATHER>
__global__ void __launch_bounds__(64) k_p2p(PointRoles R, const int32_t *__restrict__ leaves,
                                            const int32_t *__restrict__ uptr,
                                            const int32_t *__restrict__ uidx, P2PGather gs,
                                            const double *__restrict__ q, int nbatch, int bt0,
                                            const double2 *__restrict__ logtab, double *__restrict__ acc) {
    constexpr int CAP = P2PCap<NB>::value;
    // the source tile lives in the logarithm table's unused entries when it fits
    constexpr int SRC = (2 + NB) * CAP;  // doubles: x, y, q per density
    constexpr bool IN_GAP = SRC * 8 <= (LOG_BASE - 1) * 16;
    __shared__ double2 ltab[LOG_BASE + LOG_TABLE + (IN_GAP ? 0 : (SRC + 1) / 2)];
    double *xs = reinterpret_cast<double *>(IN_GAP ? ltab + 1 : ltab + LOG_BASE + LOG_TABLE);
    double *ys = xs + CAP;
    double(*qs)[CAP] = reinterpret_cast<double(*)[CAP]>(ys + CAP);
    if (!GRAD) {
        for (int i = threadIdx.x; i < LOG_TABLE; i += 64) ltab[LOG_BASE + i] = logtab[i];
        if (threadIdx.x == 0) ltab[0] = make_double2(0.0, log2p1_over_u(-1.0));
    }
    __shared__ double red[GRAD ? 2 * NB : NB][64];
    const int lane = threadIdx.x;
    const int b = leaves[blockIdx.x];
    const int t0 = R.tb[b], t1 = R.te[b];
    if (t1 <= t0) return;
    const int nt = t1 - t0;
    const int T2 = nt < 64 ? nt : 64;  // lanes per group: one target each
    const int K = 64 / T2;             // groups, each taking every K-th source
    const int tl = lane % T2, kg = lane / T2;
    const int nbh = min(NB, nbatch - bt0);
    const int e0 = uptr[b], e1 = uptr[b + 1];
    for (int base = t0; base < t1; base += 64) {
        const int t = base + tl;
        const bool act = t < t1 && kg < K;
        const double px = act ? R.tx[t] : 0.0, py = act ? R.ty[t] : 0.0;
        double a[NB], gxa[NB], gya[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) a[k] = gxa[k] = gya[k] = 0.0;
        int e = e0, eoff = 0;
        int64_t gp = GATHER ? gs.ptr[blockIdx.x] : 0;
        const int64_t gend = GATHER ? gs.ptr[blockIdx.x + 1] : 0;
        while (GATHER ? gp < gend : e < e1) {
            // fill one tile from the list, continuing inside a leaf if needed
            __syncthreads();
            int fill = 0;
            if (GATHER) {
                // sources gathered at plan time: contiguous coordinates, indexed charges
                fill = (int)min((int64_t)CAP, gend - gp);
                for (int j = lane; j < fill; j += 64) {
                    xs[j] = gs.x[gp + j];
                    ys[j] = gs.y[gp + j];
                    const int sj = gs.idx[gp + j];
#pragma unroll
                    for (int k = 0; k < NB; ++k) qs[k][j] = (k < nbh) ? q[(int64_t)(bt0 + k) * R.nsrc + sj] : 0.0;
                }
                gp += fill;
            }
            while (!GATHER && e < e1 && fill < CAP) {
                const int src = uidx[e];
                const int s0 = R.sb[src] + eoff, s1 = R.se[src];
                const int take = min(s1 - s0, CAP - fill);
                for (int j = lane; j < take; j += 64) {
                    xs[fill + j] = R.sx[s0 + j];
                    ys[fill + j] = R.sy[s0 + j];
#pragma unroll
                    for (int k = 0; k < NB; ++k)
                        qs[k][fill + j] = (k < nbh) ? q[(int64_t)(bt0 + k) * R.nsrc + s0 + j] : 0.0;
                }
                fill += take;
                if (s0 + take == s1) {
                    ++e;
                    eoff = 0;
                } else {
                    eoff += take;
                }
            }
            __syncthreads();
            if (act) {
#pragma unroll 4
                for (int j = kg; j < fill; j += K) {
                    const double dx = xs[j] - px, dy = ys[j] - py;
                    const double r2 = fma(dx, dx, dy * dy);
                    if (GRAD) {
                        const bool nz = r2 > 0.0;
                        const double rr = nz ? r2 : 1.0;
                        double ir2 = __builtin_amdgcn_rcp(rr);
                        ir2 = fma(fma(-rr, ir2, 1.0), ir2, ir2);
                        ir2 = fma(fma(-rr, ir2, 1.0), ir2, ir2);
                        ir2 = nz ? ir2 : 0.0;
#pragma unroll
                        for (int k = 0; k < NB; ++k) {
                            const double c = qs[k][j] * ir2;
                            gxa[k] = fma(c, dx, gxa[k]);
                            gya[k] = fma(c, dy, gya[k]);
                        }
                    } else {
                        // a zero distance gives exactly zero (see vp_log2_tab)
                        const double lg = vp_log2_tab(r2, ltab);
#pragma unroll
                        for (int k = 0; k < NB; ++k) a[k] = fma(qs[k][j], lg, a[k]);
                    }
                }
            }
        }
        // combine the K lane groups in a fixed order
        if (K > 1) {
            __syncthreads();
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if (GRAD) {
                    red[2 * k][lane] = gxa[k];
                    red[2 * k + 1][lane] = gya[k];
                } else {
                    red[k][lane] = a[k];
                }
            }
            __syncthreads();
            if (kg == 0) {
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    double s0 = 0.0, s1 = 0.0;
                    for (int g2 = 0; g2 < K; ++g2) {
                        if (GRAD) {
                            s0 += red[2 * k][g2 * T2 + tl];
                            s1 += red[2 * k + 1][g2 * T2 + tl];
                        } else {
                            s0 += red[k][g2 * T2 + tl];
                        }
                    }
                    if (GRAD) {
                        gxa[k] = s0;
                        gya[k] = s1;
                    } else {
                        a[k] = s0;
                    }
                }
            }
        }
        if (act && kg == 0) {
            for (int k = 0; k < nbh; ++k) {
                if (GRAD) {
                    acc[((int64_t)(bt0 + k) * 2 + 0) * R.ntgt + t] = INV_2PI * gxa[k];
                    acc[((int64_t)(bt0 + k) * 2 + 1) * R.ntgt + t] = INV_2PI * gya[k];
                } else if (ACCUM) {
                    acc[(int64_t)(bt0 + k) * R.ntgt + t] += -LN2_4PI * a[k];
                } else {
                    acc[(int64_t)(bt0 + k) * R.ntgt + t] = -LN2_4PI * a[k];
                }
            }
        }
        if (T2 < 64) break;  // all targets of the leaf handled in one pass
    }
}

// ----------------------------------------------------------------------------
// finish: out[b][i] = scale_i * acc[b][inv[i]] + sum_{q in row i} val[q] f[b][col[q]]
// (the sparse correction apply of Section 4 fused with the un-permutation).
// Sixteen lanes share a row, so a wave keeps four rows in flight; a row
// whose columns are one contiguous run (a cell's own nodes) reads only
// its run start instead of a column index per non-zero.  Reductions run in
// a fixed lane order.
// ----------------------------------------------------------------------------
typedef double vp_d2 __attribute__((ext_vector_type(2)));

template <int NBG, bool RUNS>
__global__ void __launch_bounds__(256) k_corr(int64_t nrows, int nbatch, int bt0, int64_t nnz,
                                              const int64_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ colv,
                                              const int32_t *__restrict__ run_start,
                                              const double *__restrict__ valv,
                                              const double *__restrict__ f, int64_t flen,
                                              double *__restrict__ out) {
    // out[b][i] = sum_{q in row i} val[q] f[b][col[q]] (nnz >= 1).  16 lanes
    // per row; a group takes R consecutive rows.  Values stream as aligned
    // pairs (16-byte non-temporal loads; the value array is padded to an even
    // length with zeros): lane l of a row reads pairs l and l + 16 from the
    // pair holding the row's first value, i.e. values [p0 & ~1, (p0 & ~1) + 64);
    // longer rows continue in a loop.  Indices are clamped to valid entries
    // and terms outside the row are multiplied by zero, so no load sits
    // behind a branch; the next rows' extents are fetched while this row's
    // values load.  With RUNS every row's columns are one contiguous run and
    // the column array is never read.  A non-finite value makes its row (or,
    // in f, every potential) non-finite either way.
    constexpr int R = NBG >= 4 ? 1 : (NBG == 2 ? 2 : 4);  // registers: R x 4 values and R x NBG sums
    const int l16 = threadIdx.x & 15;
    const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) >> 4;
    const int nbg = min(NBG, nbatch - bt0);
    const int64_t npair = (nnz + 1) >> 1;
    const vp_d2 *__restrict__ vp2 = reinterpret_cast<const vp_d2 *>(valv);
    // lane r < R fetches the extent of row base + r (clamped to a valid row)
    int64_t mp0 = 0, mp1 = 0;
    int32_t mrs = 0;
    auto fetch = [&](int64_t base) {
        const int64_t im = min(base + (l16 < R ? l16 : 0), nrows - 1);
        mp0 = rowptr[im];
        mp1 = rowptr[im + 1];
        if (RUNS) mrs = run_start[im];
    };
    int64_t i0 = grp * R;
    if (i0 < nrows) fetch(i0);
    for (; i0 < nrows; i0 += ngrp * R) {
        const int64_t im = i0 + l16;
        const bool mrow = l16 < R && im < nrows;
        int64_t p0[R], p1[R];
        int32_t rs[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool rv = i0 + r < nrows;  // rows past the end are empty
            p0[r] = __shfl(mp0, r, 16);
            p1[r] = rv ? __shfl(mp1, r, 16) : p0[r];
            rs[r] = __shfl(mrs, r, 16);
        }
        fetch(i0 + ngrp * R);  // the next rows' extents, in flight with the values
        double v[R][4];
        int32_t c[R][4];  // column indices (< 2^31, the f length)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t a0 = p0[r] & ~(int64_t)1;
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int64_t pi = (a0 >> 1) + l16 + 16 * u;
                const vp_d2 w = __builtin_nontemporal_load(vp2 + min(pi, npair - 1));  // streamed once
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int64_t qi = 2 * pi + e;
                    const bool in = qi >= p0[r] && qi < p1[r];
                    v[r][2 * u + e] = w[e] * (in ? 1.0 : 0.0);
                    c[r][2 * u + e] = RUNS ? (in ? rs[r] + (int32_t)(qi - p0[r]) : 0)
                                           : (in ? colv[min(qi, nnz - 1)] : 0);
                }
            }
        }
        double part[R][NBG];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < NBG; ++k) {
                // densities past nbg read a valid row and are never stored
                const double *fk = f + (int64_t)(bt0 + min(k, nbg - 1)) * flen;
                double a = 0.0;
#pragma unroll
                for (int u = 0; u < 4; ++u) a = fma(v[r][u], fk[c[r][u]], a);
                part[r][k] = a;
            }
        // rows reaching past the first 64 values of their pair range
#pragma unroll
        for (int r = 0; r < R; ++r) {
            for (int64_t pb = (p0[r] & ~(int64_t)1) + 64; pb < p1[r]; pb += 32) {
                const int64_t pi = (pb >> 1) + l16;
                if (2 * pi < p1[r]) {
                    const vp_d2 w = __builtin_nontemporal_load(vp2 + min(pi, npair - 1));
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const int64_t qi = 2 * pi + e;
                        const bool in = qi < p1[r];
                        const double vv = w[e] * (in ? 1.0 : 0.0);
                        const int32_t cc = RUNS ? (in ? rs[r] + (int32_t)(qi - p0[r]) : 0)
                                                : (in ? colv[min(qi, nnz - 1)] : 0);
#pragma unroll
                        for (int k = 0; k < NBG; ++k)
                            part[r][k] = fma(vv, f[(int64_t)(bt0 + min(k, nbg - 1)) * flen + cc], part[r][k]);
                    }
                }
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < NBG; ++k) {
                double t = part[r][k];
#pragma unroll
                for (int off = 8; off >= 1; off >>= 1) t += __shfl_xor(t, off, 16);
                part[r][k] = t;
            }
        // lane r writes row i0 + r
        if (mrow) {
#pragma unroll
            for (int k = 0; k < NBG; ++k) {
                double pr = 0.0;
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (r == l16) pr = part[r][k];
                if (k < nbg) out[(int64_t)(bt0 + k) * nrows + im] = pr;
            }
        }
    }
}

// The correction apply for a matrix made of cells (consecutive rows sharing
// one column run of at most 64): one wave per cell, lane = column, so a row
// is one contiguous 8-byte-per-lane load and the cell's densities stay in
// registers (no per-value gather of f).  R rows are loaded together; their
// sums across the 64 lanes use a butterfly: at each step a lane keeps half
// of its rows and adds its partner's share of them, then the remaining
// lanes of each row are summed (a fixed order: deterministic).
template <int NBG>
__global__ void __launch_bounds__(256) k_corr_cells(int ncell, const int32_t *__restrict__ cell_row,
                                                    const int32_t *__restrict__ cell_col,
                                                    const int64_t *__restrict__ cell_vb, int nbatch, int bt0,
                                                    const int64_t *__restrict__ rowptr,
                                                    const double *__restrict__ valv,
                                                    const double *__restrict__ f, int64_t flen, int64_t nrows,
                                                    double *__restrict__ out) {
    constexpr int R = 4;  // rows per batch (R x NBG sums in registers; fewer shuffles per row)
    const int lane = threadIdx.x & 63;
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const int nbg = min(NBG, nbatch - bt0);
    for (int64_t cc = w; cc < ncell; cc += nw) {
        const int r0 = cell_row[cc], r1 = cell_row[cc + 1], c0 = cell_col[cc];
        const int64_t vb = cell_vb[cc];  // this cell's values, or an identical block's
        if (vb < 0) continue;              // applied with its group by k_corr_group
        const int len = (int)(rowptr[r0 + 1] - rowptr[r0]);
        if (NBG >= 4 && len == 64) {
            // several densities: per cell U = V F, V the cell's rows x 64 values
            // and F its 64 columns x (up to 16) densities, on the matrix cores
            // in 16-row blocks (A = V rows, B = F, k = 4 s + lane/16)
            typedef Mfma<double> M;
            const int cl = lane & 15, g = lane >> 4;
            double bf[16];
            const double *fp = f + (int64_t)(bt0 + min(cl, nbg - 1)) * flen + c0 + g;
#pragma unroll
            for (int s = 0; s < 16; ++s) bf[s] = fp[4 * s];
            for (int rb0 = r0; rb0 < r1; rb0 += 16) {
                const double *vp = valv + vb + (int64_t)(min(rb0 + cl, r1 - 1) - r0) * 64 + g;
                double av[16];
#pragma unroll
                for (int s = 0; s < 16; ++s) av[s] = vp[4 * s];
                M::acc_t acc = M::zero();
#pragma unroll
                for (int s = 0; s < 16; ++s) acc = M::op(av[s], bf[s], acc);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = rb0 + M::row(i, g);
                    if (row < r1 && cl < nbg) out[(int64_t)(bt0 + cl) * nrows + row] = acc[i];
                }
            }
            continue;
        }
        if (NBG == 1 && len == 64 && (vb & 1) == 0) {
            // 64-column cells with 16-byte aligned values (the box cells): a
            // half-wave per row, each lane two adjacent columns, so one load
            // instruction moves two rows (1 KB) and eight are in flight
            const int h = lane >> 5, cl = lane & 31;
            const double f0 = f[(int64_t)bt0 * flen + c0 + 2 * cl], f1 = f[(int64_t)bt0 * flen + c0 + 2 * cl + 1];
            for (int i = r0; i < r1; i += 16) {
                double p[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int row = min(i + 2 * j + h, r1 - 1);
                    const vp_d2 v = __builtin_nontemporal_load(
                        reinterpret_cast<const vp_d2 *>(valv + vb + (int64_t)(row - r0) * 64) + cl);
                    p[j] = v.x * f0 + v.y * f1;
                }
                // sums over the 32 lanes of each half: three halving steps
                // (bits 16, 8, 4) leave one row per lane, two more add it up
                int m = 8;
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const int bit = 16 >> b;
                    const bool hi = (lane & bit) != 0;
                    m >>= 1;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if (j < m) {
                            const double keep = hi ? p[m + j] : p[j];
                            const double give = hi ? p[j] : p[m + j];
                            p[j] = keep + __shfl_xor(give, bit, 64);
                        }
                    }
                }
                double t = p[0];
                t += __shfl_xor(t, 2, 64);
                t += __shfl_xor(t, 1, 64);
                // lane's row pair index: bits 4, 3, 2 of the lane, high bit first
                const int jj = ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
                const int row = i + 2 * jj + h;
                if ((lane & 3) == 0 && row < r1) out[(int64_t)bt0 * nrows + row] = t;
            }
            continue;
        }
        const bool inc = lane < len;
        double fc[NBG];
#pragma unroll
        for (int k = 0; k < NBG; ++k)
            fc[k] = inc ? f[(int64_t)(bt0 + min(k, nbg - 1)) * flen + c0 + lane] : 0.0;
        for (int i = r0; i < r1; i += R) {
            double p[NBG][R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int row = min(i + r, r1 - 1);
                const double v =
                    __builtin_nontemporal_load(valv + vb + (int64_t)(row - r0) * len + (inc ? lane : 0));
#pragma unroll
                for (int k = 0; k < NBG; ++k) p[k][r] = v * fc[k];  // fc is zero past the run
            }
#pragma unroll
            for (int k = 0; k < NBG; ++k) {
                int m = R;
#pragma unroll
                for (int b = 0; (1 << b) < R; ++b) {
                    const int bit = 32 >> b;
                    const bool hi = (lane & bit) != 0;
                    m >>= 1;
#pragma unroll
                    for (int j = 0; j < R / 2; ++j) {
                        if (j < m) {
                            const double keep = hi ? p[k][m + j] : p[k][j];
                            const double give = hi ? p[k][j] : p[k][m + j];
                            p[k][j] = keep + __shfl_xor(give, bit, 64);
                        }
                    }
                }
                double t = p[k][0];
#pragma unroll
                for (int bit = 32 / R; bit >= 1; bit >>= 1) t += __shfl_xor(t, bit, 64);
                p[k][0] = t;
            }
            // lane's row: lane bits 5, 4, .. (one per butterfly step), high bit first
            int rr = 0;
#pragma unroll
            for (int b = 0; (1 << b) < R; ++b) rr = rr * 2 + ((lane >> (5 - b)) & 1);
            if ((lane & (64 / R - 1)) == 0 && i + rr < r1) {
#pragma unroll
                for (int k = 0; k < NBG; ++k)
                    if (k < nbg) out[(int64_t)(bt0 + k) * nrows + i + rr] = p[k][0];
            }
        }
    }
}

// out[b][i] += scale_i * (acc[b][inv[i]] + acc2[b][inv[i]]): the near- and
// far-field sums (sorted order; acc2 may be null) added to the correction
// already in out (user order)
__global__ void k_add_acc(int64_t nrows, int nbatch, const int32_t *__restrict__ inv,
                          const double *__restrict__ scale, const double *__restrict__ acc,
                          const double *__restrict__ acc2, int64_t acc_len, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    const int32_t si = inv[i];
    const double sc = scale ? scale[i] : 1.0;
    for (int b = 0; b < nbatch; ++b) {
        double *o = out + (int64_t)b * nrows + i;
        const int64_t k = (int64_t)b * acc_len + si;
        const double v = acc2 ? acc[k] + acc2[k] : acc[k];
        *o = sc * v + *o;
    }
}

// run_start[i] = first column when row i's columns are c0, c0+1, ..., else -1
__global__ void k_detect_runs(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ colv,
                              int64_t nrows, int32_t *__restrict__ run_start) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    const int64_t p0 = rowptr[i], p1 = rowptr[i + 1];
    if (p1 == p0) {
        run_start[i] = 0;
        return;
    }
    const int32_t c0 = colv[p0];
    bool run = true;
    for (int64_t q = p0 + 1; q < p1 && run; ++q) run = colv[q] == c0 + (int32_t)(q - p0);
    run_start[i] = run ? c0 : -1;
}

void build_cells(vp_plan_s *P, bool transposed);
// One density, cells sharing one value block (the box corrections of one box
// size, Section 4): U = V [f_1 .. f_16] for up to 16 such cells per wave, on
// the matrix cores in 16-row blocks; V (rows x 64) is read once per group.
// grp_cell[16 g + j] is the j-th cell of group g (-1: none); every cell of a
// group has grp_rows[g] rows of 64 columns and reads the values at grp_vb[g].
__global__ void __launch_bounds__(256) k_corr_group(int ngrp, const int32_t *__restrict__ grp_cell,
                                                    const int64_t *__restrict__ grp_vb,
                                                    const int32_t *__restrict__ grp_rows,
                                                    const int32_t *__restrict__ cell_row,
                                                    const int32_t *__restrict__ cell_col,
                                                    const double *__restrict__ valv,
                                                    const double *__restrict__ f, double *__restrict__ out) {
    typedef Mfma<double> M;
    const int lane = threadIdx.x & 63, cl = lane & 15, g = lane >> 4;
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t gi = w; gi < ngrp; gi += nw) {
        const int cell = grp_cell[gi * 16 + cl];
        const int R = grp_rows[gi];
        const int64_t vb = grp_vb[gi];
        // B = F: column cl holds f at cell `cell`'s 64 columns, k = 4 s + lane/16
        double bf[16];
        int r0 = 0;
        if (cell >= 0) {
            r0 = cell_row[cell];
            const double *fp = f + cell_col[cell] + g;
#pragma unroll
            for (int s = 0; s < 16; ++s) bf[s] = fp[4 * s];
        } else {
#pragma unroll
            for (int s = 0; s < 16; ++s) bf[s] = 0.0;
        }
        for (int rb = 0; rb < R; rb += 16) {
            const double *vp = valv + vb + (int64_t)min(rb + cl, R - 1) * 64 + g;
            double av[16];
#pragma unroll
            for (int s = 0; s < 16; ++s) av[s] = vp[4 * s];
            M::acc_t acc = M::zero();
#pragma unroll
            for (int s = 0; s < 16; ++s) acc = M::op(av[s], bf[s], acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = rb + M::row(i, g);
                if (row < R && cell >= 0) out[r0 + row] = acc[i];
            }
        }
    }
}


// Plan time: a 64-bit fingerprint of each cell's value block (one wave per
// cell; every value's bits mixed with its position, xor over the block).
__device__ inline uint64_t vp_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__global__ void __launch_bounds__(256) k_cell_hash(int ncell, const int32_t *__restrict__ cell_row,
                                                   const int64_t *__restrict__ rowptr,
                                                   const double *__restrict__ val, uint64_t *__restrict__ hash) {
    const int lane = threadIdx.x & 63;
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t cc = w; cc < ncell; cc += nw) {
        const int64_t v0 = rowptr[cell_row[cc]], v1 = rowptr[cell_row[cc + 1]];
        uint64_t h = 0;
        for (int64_t e = v0 + lane; e < v1; e += 64)
            h ^= vp_mix64((uint64_t)__double_as_longlong(val[e]) + (uint64_t)(e - v0) * 0x9e3779b97f4a7c15ull);
        for (int b = 32; b >= 1; b >>= 1) h ^= (uint64_t)__shfl_xor((unsigned long long)h, b, 64);
        if (lane == 0) hash[cc] = h ^ vp_mix64((uint64_t)(v1 - v0));
    }
}
// Plan time: same[i] = 1 when candidate cell cand[i] holds exactly the
// values of cell rep[i] (same length, bit for bit)
__global__ void __launch_bounds__(256) k_cell_same(int ncand, const int32_t *__restrict__ cand,
                                                   const int32_t *__restrict__ rep,
                                                   const int32_t *__restrict__ cell_row,
                                                   const int64_t *__restrict__ rowptr,
                                                   const double *__restrict__ val, int32_t *__restrict__ same) {
    const int lane = threadIdx.x & 63;
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t i = w; i < ncand; i += nw) {
        const int64_t a0 = rowptr[cell_row[cand[i]]], a1 = rowptr[cell_row[cand[i] + 1]];
        const int64_t b0 = rowptr[cell_row[rep[i]]], b1 = rowptr[cell_row[rep[i] + 1]];
        bool eq = (a1 - a0) == (b1 - b0);
        for (int64_t e = lane; eq && e < a1 - a0; e += 64)
            eq = __double_as_longlong(val[a0 + e]) == __double_as_longlong(val[b0 + e]);
        const bool all = __all(eq);
        if (lane == 0) same[i] = all ? 1 : 0;
    }
}

void detect_runs(vp_plan_s *P) {
    hipStream_t s = P->stream;
    P->run_start = P->mem.alloc<int32_t>(P->m);
    // the transpose has one row per density value (nd)
    P->run_startT = P->mem.alloc<int32_t>(P->nd);
    hipLaunchKernelGGL(k_detect_runs, dim3((unsigned)((P->m + 255) / 256)), dim3(256), 0, s, P->rowptr, P->col, P->m,
                       P->run_start);
    hipLaunchKernelGGL(k_detect_runs, dim3((unsigned)((P->nd + 255) / 256)), dim3(256), 0, s, P->rowptrT, P->colT,
                       P->nd, P->run_startT);
    VP_LAUNCH_CHECK();
    // every row a run: the apply kernel never reads the column array
    std::vector<int32_t> h(std::max(P->m, P->nd));
    VP_HIP(hipMemcpyAsync(h.data(), P->run_start, 4 * P->m, hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));
    P->all_runs = std::all_of(h.begin(), h.begin() + P->m, [](int32_t v) { return v >= 0; });
    VP_HIP(hipMemcpyAsync(h.data(), P->run_startT, 4 * P->nd, hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));
    P->all_runsT = std::all_of(h.begin(), h.begin() + P->nd, [](int32_t v) { return v >= 0; });
    build_cells(P, false);
    build_cells(P, true);
}

// Cells of a run-structured matrix: maximal groups of consecutive rows whose
// columns are the same run of at most 64 (a cell's own nodes, for the
// own-cell corrections of Section 4).  Used when the cells average at least
// 8 rows; otherwise (or when some row is not such a run) the row kernel
// applies the matrix.
void build_cells(vp_plan_s *P, bool transposed) {
    hipStream_t s = P->stream;
    const int64_t nrows = transposed ? P->nd : P->m;
    const bool runs = transposed ? P->all_runsT : P->all_runs;
    int32_t *&cell_row = transposed ? P->cell_rowT : P->cell_row;
    int32_t *&cell_col = transposed ? P->cell_colT : P->cell_col;
    int &ncell = transposed ? P->ncellT : P->ncell;
    ncell = 0;
    if (!runs || P->nnz == 0 || nrows >= (int64_t)1 << 31) return;
    std::vector<int64_t> rp(nrows + 1);
    std::vector<int32_t> rs(nrows);
    VP_HIP(hipMemcpyAsync(rp.data(), transposed ? P->rowptrT : P->rowptr, 8 * (nrows + 1), hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(rs.data(), transposed ? P->run_startT : P->run_start, 4 * nrows, hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> row0, col0;
    for (int64_t i = 0; i < nrows; ++i) {
        const int64_t len = rp[i + 1] - rp[i];
        if (len > 64) return;
        if (i == 0 || rs[i] != rs[i - 1] || len != rp[i] - rp[i - 1]) {
            row0.push_back((int32_t)i);
            col0.push_back(rs[i]);
        }
    }
    if ((int64_t)row0.size() * 8 > nrows) return;
    row0.push_back((int32_t)nrows);
    cell_row = P->mem.alloc<int32_t>(row0.size());
    cell_col = P->mem.alloc<int32_t>(col0.size());
    VP_HIP(hipMemcpyAsync(cell_row, row0.data(), 4 * row0.size(), hipMemcpyHostToDevice, s));
    VP_HIP(hipMemcpyAsync(cell_col, col0.data(), 4 * col0.size(), hipMemcpyHostToDevice, s));
    const int nc = (int)col0.size();
    // cells with identical value blocks (the box corrections of one box size
    // are one lookup table, Section 4): each reads the first such cell's
    // values, which then stay in the caches; found by fingerprint, then
    // confirmed bit for bit on the device
    const double *vv = transposed ? P->valT : P->val;
    const int64_t *rpd = transposed ? P->rowptrT : P->rowptr;
    uint64_t *dh = P->mem.alloc<uint64_t>(nc);
    const unsigned hb = (unsigned)std::min<int64_t>((nc + 3) / 4, 16384);
    hipLaunchKernelGGL(k_cell_hash, dim3(hb), dim3(256), 0, s, nc, cell_row, rpd, vv, dh);
    VP_LAUNCH_CHECK();
    std::vector<uint64_t> hh(nc);
    VP_HIP(hipMemcpyAsync(hh.data(), dh, 8 * (size_t)nc, hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> vbh(nc);
    for (int k = 0; k < nc; ++k) vbh[k] = rp[row0[k]];
    std::unordered_map<uint64_t, int> first;
    std::vector<int32_t> cand, rep;
    for (int k = 0; k < nc; ++k) {
        const int rows = row0[k + 1] - row0[k];
        const uint64_t key = hh[k] ^ ((uint64_t)rows * 0x9e3779b97f4a7c15ull);
        auto it = first.find(key);
        if (it == first.end()) first.emplace(key, k);
        else {
            cand.push_back(k);
            rep.push_back(it->second);
        }
    }
    int nshared = 0;
    int64_t nread = P->nnz;
    if (!cand.empty()) {
        int32_t *dc = P->mem.alloc<int32_t>(cand.size()), *dr = P->mem.alloc<int32_t>(rep.size());
        int32_t *ds = P->mem.alloc<int32_t>(cand.size());
        VP_HIP(hipMemcpyAsync(dc, cand.data(), 4 * cand.size(), hipMemcpyHostToDevice, s));
        VP_HIP(hipMemcpyAsync(dr, rep.data(), 4 * rep.size(), hipMemcpyHostToDevice, s));
        const unsigned sb = (unsigned)std::min<int64_t>(((int64_t)cand.size() + 3) / 4, 16384);
        hipLaunchKernelGGL(k_cell_same, dim3(sb), dim3(256), 0, s, (int)cand.size(), dc, dr, cell_row, rpd, vv, ds);
        VP_LAUNCH_CHECK();
        std::vector<int32_t> same(cand.size());
        VP_HIP(hipMemcpyAsync(same.data(), ds, 4 * same.size(), hipMemcpyDeviceToHost, s));
        VP_HIP(hipStreamSynchronize(s));
        for (size_t i = 0; i < cand.size(); ++i)
            if (same[i]) {
                vbh[cand[i]] = rp[row0[rep[i]]];
                ++nshared;
                nread -= rp[row0[cand[i] + 1]] - rp[row0[cand[i]]];
            }
    }
    int64_t *&cvb = transposed ? P->cell_vbT : P->cell_vb;
    cvb = P->mem.alloc<int64_t>(nc);
    VP_HIP(hipMemcpyAsync(cvb, vbh.data(), 8 * (size_t)nc, hipMemcpyHostToDevice, s));
    // every cell a 64 x 64 block reading one shared block (uniform grids: the
    // box corrections of one box size): C is one fixed operator applied to
    // every (cell, density) column, the fixed-operator kernel's case
    {
        bool one = nc > 0;
        for (int k = 0; one && k < nc; ++k)
            one = row0[k + 1] - row0[k] == 64 && rp[row0[k] + 1] - rp[row0[k]] == 64 && vbh[k] == vbh[0];
        double *&op = transposed ? P->corr_opT : P->corr_op;
        op = nullptr;
        if (one) {
            std::vector<double> A(64 * 64), F(64 * 64);
            VP_HIP(hipMemcpyAsync(A.data(), vv + vbh[0], 8 * A.size(), hipMemcpyDeviceToHost, s));
            VP_HIP(hipStreamSynchronize(s));
            vp_to_frag(A.data(), 64, 64, 64, F.data());  // rows = cell rows, cols = the cell's column run
            if (!transposed) {
                P->corr_block = A;
                P->corr_cell_row = row0;
                P->corr_cell_col = col0;
            }
            op = P->mem.alloc<double>(F.size());
            VP_HIP(hipMemcpyAsync(op, F.data(), 8 * F.size(), hipMemcpyHostToDevice, s));
            if (!P->cell_iota || (int)P->n_cell_iota < nc) {
                std::vector<int32_t> io(nc);
                for (int k = 0; k < nc; ++k) io[k] = k;
                P->cell_iota = P->mem.alloc<int32_t>(nc);
                P->n_cell_iota = nc;
                VP_HIP(hipMemcpyAsync(P->cell_iota, io.data(), 4 * (size_t)nc, hipMemcpyHostToDevice, s));
            }
            VP_HIP(hipStreamSynchronize(s));  // A, F and io leave scope
        }
    }
    // one density: 64-column cells reading one block, at least 8 of them,
    // go to k_corr_group in groups of 16; the cell kernel skips them (-1)
    std::map<std::pair<int64_t, int>, std::vector<int32_t>> bykey;
    for (int k = 0; k < nc; ++k) {
        const int rows = row0[k + 1] - row0[k];
        if (rows > 0 && rp[row0[k] + 1] - rp[row0[k]] == 64) bykey[{vbh[k], rows}].push_back(k);
    }
    std::vector<int64_t> vbg(vbh), gvb;
    std::vector<int32_t> gcell, grows;
    for (auto &kv : bykey) {
        if (kv.second.size() < 8) continue;
        for (size_t i = 0; i < kv.second.size(); i += 16) {
            for (size_t j = i; j < i + 16; ++j) {
                const int32_t k = j < kv.second.size() ? kv.second[j] : -1;
                gcell.push_back(k);
                if (k >= 0) vbg[k] = -1;
            }
            gvb.push_back(kv.first.first);
            grows.push_back(kv.first.second);
        }
    }
    int &ng = transposed ? P->ngrpT : P->ngrp;
    ng = (int)gvb.size();
    if (ng > 0) {
        int64_t *&cvbg = transposed ? P->cell_vbgT : P->cell_vbg;
        int32_t *&gc = transposed ? P->grp_cellT : P->grp_cell;
        int64_t *&gv = transposed ? P->grp_vbT : P->grp_vb;
        int32_t *&gr = transposed ? P->grp_rowsT : P->grp_rows;
        cvbg = P->mem.alloc<int64_t>(nc);
        gc = P->mem.alloc<int32_t>(gcell.size());
        gv = P->mem.alloc<int64_t>(ng);
        gr = P->mem.alloc<int32_t>(ng);
        VP_HIP(hipMemcpyAsync(cvbg, vbg.data(), 8 * (size_t)nc, hipMemcpyHostToDevice, s));
        VP_HIP(hipMemcpyAsync(gc, gcell.data(), 4 * gcell.size(), hipMemcpyHostToDevice, s));
        VP_HIP(hipMemcpyAsync(gv, gvb.data(), 8 * (size_t)ng, hipMemcpyHostToDevice, s));
        VP_HIP(hipMemcpyAsync(gr, grows.data(), 4 * (size_t)ng, hipMemcpyHostToDevice, s));
    }
    VP_HIP(hipStreamSynchronize(s));  // host vectors leave scope
    if (!transposed) {
        P->ncell_shared = nshared;
        P->corr_values_read = nread;
    }
    ncell = nc;
}

__global__ void k_unpermute_grad(int64_t m, int nbatch, const int32_t *__restrict__ inv,
                                 const double *__restrict__ acc, double *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int32_t si = inv[i];
    for (int bt = 0; bt < nbatch; ++bt)
        for (int d = 0; d < 2; ++d)
            out[((int64_t)bt * 2 + d) * m + i] = acc[((int64_t)bt * 2 + d) * m + si];
}

// ----------------------------------------------------------------------------
// Schedules (plan time): box groups for each pass.
// ----------------------------------------------------------------------------
std::vector<P2MJob> p2m_job_descs(vp_plan_s *P, const std::vector<int32_t> &codes, bool target_role) {
    Tree &T = P->tree;
    hipStream_t s = P->stream;
    const int nbox = T.nbox, nv = P->n_vleaf;
    std::vector<int32_t> lev(nbox), b0(nbox), b1(nbox), vl(nv), vs(5 * (size_t)nv);
    std::vector<double> cx(nbox), cy(nbox);
    VP_HIP(hipMemcpyAsync(lev.data(), T.level, 4 * (size_t)nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(b0.data(), target_role ? T.tb : T.sb, 4 * (size_t)nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(b1.data(), target_role ? T.te : T.se, 4 * (size_t)nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(cx.data(), T.cx, 8 * (size_t)nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(cy.data(), T.cy, 8 * (size_t)nbox, hipMemcpyDeviceToHost, s));
    if (nv > 0) {
        VP_HIP(hipMemcpyAsync(vl.data(), P->vleaf, 4 * (size_t)nv, hipMemcpyDeviceToHost, s));
        VP_HIP(hipMemcpyAsync(vs.data(), target_role ? P->vsplit_t : P->vsplit_s, 4 * vs.size(),
                              hipMemcpyDeviceToHost, s));
    }
    VP_HIP(hipStreamSynchronize(s));
    std::vector<P2MJob> out(codes.size());
    for (size_t i = 0; i < codes.size(); ++i) {
        const int c = codes[i];
        P2MJob &j = out[i];
        j.pad = 0;
        if (c >= 0) {
            j.cx = cx[c];
            j.cy = cy[c];
            j.inv_s = 1.0 / T.side[lev[c]];
            j.s0 = b0[c];
            j.s1 = b1[c];
            j.col = c;
        } else {
            const int vq = ~c, v = vq >> 2, qd = vq & 3, a = vl[v];
            const double h = T.side[lev[a]];
            j.cx = cx[a] + ((qd & 1) ? 0.25 : -0.25) * h;
            j.cy = cy[a] + ((qd >> 1) ? 0.25 : -0.25) * h;
            j.inv_s = 2.0 / h;
            j.s0 = vs[5 * (size_t)v + qd];
            j.s1 = vs[5 * (size_t)v + qd + 1];
            j.col = nbox + vq;
        }
    }
    return out;
}

std::vector<int32_t> tile_order_by_work(const std::vector<int32_t> &tile_ptr, int group) {
    const int nt = (int)tile_ptr.size() - 1;
    std::vector<int32_t> ord(std::max(nt, 0));
    for (int t = 0; t < nt; ++t) ord[t] = t;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) {
        return tile_ptr[x + 1] - tile_ptr[x] > tile_ptr[y + 1] - tile_ptr[y];
    });
    // The chip deals workgroup b to XCD b % 8, and each XCD has its own L2.
    // Dealt one by one, consecutive tiles (neighbouring boxes, which share
    // most of their source columns) land on eight different L2s and every
    // source column is fetched past L2 once per target.  Instead each XCD
    // takes runs of XCD_RUN consecutive workgroups' tiles (a workgroup takes
    // `group` consecutive tiles of the order above): round r covers
    // workgroups [8 r XCD_RUN, 8 (r+1) XCD_RUN), XCD x its x-th run, so the
    // order's heaviest-first progress is kept round by round.  The last,
    // incomplete round (and a last, partial workgroup) keep the plain order.
    constexpr int XCDS = 8, XCD_RUN = 256;
    const int nu = (nt + group - 1) / group;         // workgroups
    const int nfull = nt / group;                    // workgroups with `group` tiles
    const int full = nfull / (XCDS * XCD_RUN) * (XCDS * XCD_RUN);
    std::vector<int32_t> launch(ord.size());
    for (int p = 0; p < nu; ++p) {
        int b = p;
        if (p < full) {
            const int run = p / XCD_RUN, x = run % XCDS, round = run / XCDS;
            const int j = round * XCD_RUN + p % XCD_RUN;  // position in XCD x's sequence
            b = j * XCDS + x;
        }
        for (int w = 0; w < group && p * group + w < nt; ++w) launch[(size_t)b * group + w] = ord[(size_t)p * group + w];
    }
    return launch;
}

void build_schedules(vp_plan_s *P) {
    Tree &T = P->tree;
    hipStream_t s = P->stream;
    const int nbox = T.nbox;
    std::vector<int32_t> lev(nbox), ix(nbox), iy(nbox), nch(nbox), chb(nbox), par(nbox), xp(nbox + 1),
        wp(nbox + 1);
    VP_HIP(hipMemcpyAsync(lev.data(), T.level, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(ix.data(), T.ix, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(iy.data(), T.iy, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(nch.data(), T.nchild, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(chb.data(), T.child, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(par.data(), T.parent, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(xp.data(), T.lptr[3], 4 * (nbox + 1), hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(wp.data(), T.lptr[2], 4 * (nbox + 1), hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));
    auto up = [&](const std::vector<int32_t> &h) {
        int32_t *d = P->mem.alloc<int32_t>(h.size());
        if (!h.empty()) VP_HIP(hipMemcpyAsync(d, h.data(), 4 * h.size(), hipMemcpyHostToDevice, s));
        return d;
    };
    auto cls = [&](int b) { return (ix[b] & 1) | ((iy[b] & 1) << 1); };
    // split level: the expansion passes below it (few boxes per level, each
    // launch latency bound) run on a third stream beside the M2L of the
    // levels from it on, which hold at least 85% of the M2L columns
    {
        std::vector<int64_t> per_level(T.nlevels + 1, 0);
        int64_t total = 0;
        for (int b = 0; b < nbox; ++b)
            if (lev[b] >= 2) ++per_level[lev[b]], ++total;
        int L0 = 2;
        int64_t above = 0;
        for (int l = T.nlevels - 1; l >= 2; --l) {
            above += per_level[l];
            if (above >= (total * 85 + 99) / 100) {
                L0 = l;
                break;
            }
        }
        P->split_level = std::max(2, std::min(L0, T.nlevels - 1));
    }
    // per level: boxes grouped by class (L2L), non-leaf boxes (M2M)
    std::vector<int32_t> lb, parents;
    P->lvl_box_begin.assign(T.nlevels + 1, 0);
    P->m2m_begin.assign(T.nlevels + 1, 0);
    for (int l = 0; l < T.nlevels; ++l) {
        P->lvl_box_begin[l] = (int)lb.size();
        P->m2m_begin[l] = (int)parents.size();
        for (int c = 0; c < 4; ++c)
            for (int b = T.level_begin[l]; b < T.level_begin[l + 1]; ++b)
                if (cls(b) == c) lb.push_back(b);
        for (int b = T.level_begin[l]; b < T.level_begin[l + 1]; ++b)
            if (nch[b] > 0) parents.push_back(b);
    }
    P->lvl_box_begin[T.nlevels] = (int)lb.size();
    P->m2m_begin[T.nlevels] = (int)parents.size();
    P->lvl_boxes = up(lb);
    P->m2m_parents = up(parents);
    // beside the launch lists: each parent's child per quadrant (M2M; the
    // quadrant is the child's class), each box's parent * 4 + class (L2L)
    std::vector<int32_t> cs(parents.size() * 4, -1), pcls(lb.size(), 0);
    for (size_t k = 0; k < parents.size(); ++k) {
        const int b = parents[k];
        for (int c = chb[b]; c < chb[b] + nch[b]; ++c) cs[k * 4 + cls(c)] = c;
    }
    for (size_t k = 0; k < lb.size(); ++k) pcls[k] = par[lb[k]] >= 0 ? par[lb[k]] * 4 + cls(lb[k]) : 0;
    P->m2m_cslot = up(cs);
    P->lvl_pcls = up(pcls);
    std::vector<int32_t> p2m, xb, wl;
    for (int b = 0; b < nbox; ++b) {
        if (nch[b] == 0 && lev[b] >= 2) p2m.push_back(b);
        if (nch[b] == 0 && wp[b + 1] > wp[b]) wl.push_back(b);
    }
    // longest W lists first (they run in their own launch)
    std::stable_sort(wl.begin(), wl.end(), [&](int x, int y) { return wp[x + 1] - wp[x] > wp[y + 1] - wp[y]; });

    // X list, one level apart: the source leaf a (level l-1) splits into four
    // virtual children on the target's level l.  None of them is adjacent to
    // the target b (a is not), and they lie in b's 7x7 neighbourhood (b's
    // parent is adjacent to a), i.e. at outer offsets where the target has
    // no V-list box (a is a leaf, so no real box exists there).  Their
    // multipoles (P2M over the points of each quadrant) enter the target's
    // M2L slots; entries further apart stay on the P2L kernel.
    const int64_t nx = T.llen[3];
    std::vector<int32_t> xidx(nx), vslot((size_t)nbox * NOFF), sb(nbox), se(nbox), tb(nbox), te(nbox);
    std::vector<uint64_t> skey(P->n), tkey(P->m);
    if (nx) VP_HIP(hipMemcpyAsync(xidx.data(), T.lidx[3], 4 * nx, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(vslot.data(), T.v_slot, 4 * vslot.size(), hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(sb.data(), T.sb, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(se.data(), T.se, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(tb.data(), T.tb, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(te.data(), T.te, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(skey.data(), P->skeys, 8 * P->n, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(tkey.data(), P->tkeys, 8 * P->m, hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> vindex(nbox, -1), vleaf, vsplit_s, vsplit_t, xr_ptr(1, 0), xr_idx;
    // quadrant boundaries of a leaf's sorted points (Morton order keeps each
    // quadrant contiguous): split[0..4]
    auto splits = [&](const std::vector<uint64_t> &key, int b0, int b1, int la, std::vector<int32_t> &out) {
        const int shift = 2 * (LBITS - la - 1);
        out.push_back(b0);
        for (int qd = 1; qd < 4; ++qd) {
            int lo = b0, hi = b1;  // first index with quadrant >= qd
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if ((int)((key[mid] >> shift) & 3) < qd) lo = mid + 1;
                else hi = mid;
            }
            out.push_back(lo);
        }
        out.push_back(b1);
    };
    for (int b = 0; b < nbox; ++b) {
        for (int e = xp[b]; e < xp[b + 1]; ++e) {
            const int a = xidx[e];
            if (lev[b] - lev[a] != 1 || lev[a] + 1 > LBITS) {
                xr_idx.push_back(a);
                continue;
            }
            if (vindex[a] < 0) {
                vindex[a] = (int)vleaf.size();
                vleaf.push_back(a);
                splits(skey, sb[a], se[a], lev[a], vsplit_s);
                splits(tkey, tb[a], te[a], lev[a], vsplit_t);
            }
            const int va = vindex[a];
            for (int qd = 0; qd < 4; ++qd) {
                const int ns = vsplit_s[5 * va + qd + 1] - vsplit_s[5 * va + qd];
                const int nt = vsplit_t[5 * va + qd + 1] - vsplit_t[5 * va + qd];
                if (ns + nt == 0) continue;
                const int dx = 2 * ix[a] + (qd & 1) - ix[b], dy = 2 * iy[a] + (qd >> 1) - iy[b];
                const int code = offset_code(dx, dy);
                if (code < 0 || vslot[(size_t)b * NOFF + code] >= 0)
                    throw Error(VP_EINTERNAL, "X-list entry outside the interaction offsets");
                vslot[(size_t)b * NOFF + code] = nbox + 4 * va + qd;
            }
        }
        xr_ptr.push_back((int32_t)xr_idx.size());
        if (xr_ptr[b + 1] > xr_ptr[b]) xb.push_back(b);
    }
    P->n_vleaf = (int)vleaf.size();
    P->vleaf = up(vleaf);
    // VALU P2M jobs without tables: every leaf of level >= 2, then the four
    // virtual children of each X-list source (job ~(4 v + quadrant))
    std::vector<int32_t> p2m_jobs(p2m);
    for (int v = 0; v < (int)vleaf.size(); ++v)
        for (int qd = 0; qd < 4; ++qd) p2m_jobs.push_back(~(4 * v + qd));
    P->n_p2m_jobs = (int)p2m_jobs.size();
    P->vsplit_s = up(vsplit_s);
    P->vsplit_t = up(vsplit_t);
    VP_HIP(hipMemcpyAsync(T.v_slot, vslot.data(), 4 * vslot.size(), hipMemcpyHostToDevice, s));
    // M2L launches (levels from the split level on; levels 2 .. split - 1).
    // With fewer than 16 densities a tile holds several boxes: columns are
    // then grouped by child class (boxes of one class share their 27 V-list
    // offsets in a uniform region), within a class ordered by their set of
    // offsets (stable, so equal sets keep their tree order), so that
    // 16-column tiles share their offsets wherever the tree is not uniform.
    // A tile of one box has nothing to share: the boxes keep their tree
    // (Morton) order, in which neighbouring tiles share source columns.
    P->m2l_translations = P->m2l_tile_ops = 0;
    const bool group_class = P->nbatch < 16;
    for (int part = 0; part < 2; ++part) {
        M2LSched &S = P->m2l[part];
        std::vector<int32_t> m2l;
        for (int c = 0; c < (group_class ? 4 : 1); ++c)
            for (int b = 0; b < nbox; ++b)
                if (lev[b] >= 2 && (!group_class || cls(b) == c) && (lev[b] >= P->split_level) == (part == 0))
                    m2l.push_back(b);
        std::vector<uint64_t> omask(nbox, 0);
        for (int b : m2l)
            for (int o = 0; o < NOFF; ++o)
                if (vslot[(size_t)b * NOFF + o] >= 0) omask[b] |= 1ull << o;
        if (group_class)
            std::stable_sort(m2l.begin(), m2l.end(), [&](int x, int y) {
                const int cx = cls(x), cy = cls(y);
                return cx != cy ? cx < cy : omask[x] < omask[y];
            });
        // offsets present in each 16-column tile (columns = box x density)
        const int64_t ncols = (int64_t)m2l.size() * P->nbatch;
        const int64_t ntiles = (ncols + 15) / 16;
        std::vector<int32_t> tptr(1, 0), tops, tsrc;
        for (int64_t t = 0; t < ntiles; ++t) {
            uint64_t mask = 0;
            for (int64_t c = 16 * t; c < std::min(ncols, 16 * t + 16); ++c) mask |= omask[m2l[c / P->nbatch]];
            for (int o = 0; o < NOFF; ++o)
                if (mask >> o & 1) {
                    tops.push_back(o);
                    // each column's source box for this offset (-1: none)
                    for (int64_t c = 16 * t; c < 16 * t + 16; ++c)
                        tsrc.push_back(c < ncols ? vslot[(size_t)m2l[c / P->nbatch] * NOFF + o] : -1);
                }
            tptr.push_back((int32_t)tops.size());
        }
        const std::vector<int32_t> order = tile_order_by_work(tptr), order4 = tile_order_by_work(tptr, 4);
        S.nboxes = (int)m2l.size();
        S.tile_ops = (int64_t)tops.size();
        S.translations = 0;
        for (int b : m2l) S.translations += __builtin_popcountll(omask[b]);
        S.cols = up(m2l);
        S.tptr = up(tptr);
        S.tops = up(tops);
        S.tsrc = up(tsrc);
        S.torder = up(order);
        S.torder4 = up(order4);
        P->m2l_translations += S.translations;
        P->m2l_tile_ops += S.tile_ops;
        VP_HIP(hipStreamSynchronize(s));  // the host vectors leave scope
    }
    {
        // VALU P2M descriptors (the virtual-children tables are on the device now)
        VP_HIP(hipStreamSynchronize(s));
        const std::vector<P2MJob> ds = p2m_job_descs(P, p2m_jobs, false), dt = p2m_job_descs(P, p2m_jobs, true);
        P->p2m_jobs = P->mem.alloc<P2MJob>(ds.size());
        P->p2m_jobs_t = P->mem.alloc<P2MJob>(dt.size());
        if (!ds.empty()) {
            VP_HIP(hipMemcpyAsync(P->p2m_jobs, ds.data(), sizeof(P2MJob) * ds.size(), hipMemcpyHostToDevice, s));
            VP_HIP(hipMemcpyAsync(P->p2m_jobs_t, dt.data(), sizeof(P2MJob) * dt.size(), hipMemcpyHostToDevice, s));
        }
        VP_HIP(hipStreamSynchronize(s));  // ds, dt leave scope
    }
    P->xr_ptr = up(xr_ptr);
    P->xr_idx = up(xr_idx);
    P->n_x_boxes = (int)xb.size();
    P->x_boxes = up(xb);
    // P2L writes these boxes' local expansions first; M2L then adds to them
    std::vector<int32_t> xinit(nbox, 0);
    for (int b : xb) {
        if (lev[b] < 2) throw Error(VP_EINTERNAL, "P2L target above level 2");
        xinit[b] = 1;
    }
    P->x_init = up(xinit);
    P->n_w_leaves = (int)wl.size();
    P->w_leaves = up(wl);
    VP_HIP(hipStreamSynchronize(s));
}

// ----------------------------------------------------------------------------
// Gather-GEMM launches of the per-offset M2L form
// ----------------------------------------------------------------------------
template <class TI, class TO, class TM, bool SPLIT, int RB>
static void launch_split(hipStream_t s, int nw, const TranslateArgs &a, const TM *Ahi, const TM *Alo, const TI *in,
                         TO *out) {
    constexpr int S = RB * 4;
    const unsigned blocks = (unsigned)((a.ncols + 15) / 16);
    if (nw == 2)
        hipLaunchKernelGGL((k_translate_split<TI, TO, TM, RB, S, SPLIT, false, 2>), dim3(blocks), dim3(128), 0, s, a,
                           Ahi, Alo, in, out);
    else
        hipLaunchKernelGGL((k_translate_split<TI, TO, TM, RB, S, SPLIT, false, 4>), dim3(blocks), dim3(256), 0, s, a,
                           Ahi, Alo, in, out);
    VP_LAUNCH_CHECK();
}

// M2L: operators split across the waves of a workgroup (overwrite only)
template <class TI, class TO, class TM, bool SPLIT>
static void translate_m2l(hipStream_t s, int nw, int PD, const TranslateArgs &a, const TM *Ahi, const TM *Alo,
                          const TI *in, TO *out) {
    if (a.ncols <= 0) return;
    switch (PD) {
        case 16: launch_split<TI, TO, TM, SPLIT, 1>(s, nw, a, Ahi, Alo, in, out); break;
        case 32: launch_split<TI, TO, TM, SPLIT, 2>(s, nw, a, Ahi, Alo, in, out); break;
        case 48: launch_split<TI, TO, TM, SPLIT, 3>(s, nw, a, Ahi, Alo, in, out); break;
        case 64: launch_split<TI, TO, TM, SPLIT, 4>(s, nw, a, Ahi, Alo, in, out); break;
        case 80: launch_split<TI, TO, TM, SPLIT, 5>(s, nw, a, Ahi, Alo, in, out); break;
        case 96: launch_split<TI, TO, TM, SPLIT, 6>(s, nw, a, Ahi, Alo, in, out); break;
        case 112: launch_split<TI, TO, TM, SPLIT, 7>(s, nw, a, Ahi, Alo, in, out); break;
        case 128: launch_split<TI, TO, TM, SPLIT, 8>(s, nw, a, Ahi, Alo, in, out); break;
        default: throw Error(VP_EUNSUPPORTED, "unsupported expansion size");
    }
}

template <class TI, class TO, class TM, int RB>
static void launch_m2l_scaled(hipStream_t s, int nw, unsigned blocks, const M2LScaledArgs &a, const TM *Q,
                              const TM *tin, const double *logt, const TI *in, TO *out) {
    if (nw == 1)
        hipLaunchKernelGGL((k_m2l_wave<TI, TO, TM, RB>), dim3((blocks + 3) / 4), dim3(256), 0, s, a, Q, tin, logt,
                           in, out);
    else if (nw == 2)
        hipLaunchKernelGGL((k_m2l_scaled<TI, TO, TM, RB, 2>), dim3(blocks), dim3(128), 0, s, a, Q, tin, logt, in, out);
    else
        hipLaunchKernelGGL((k_m2l_scaled<TI, TO, TM, RB, 4>), dim3(blocks), dim3(256), 0, s, a, Q, tin, logt, in, out);
}

template <class TI, class TO, class TM>
static void m2l_scaled(hipStream_t s, int nw, int PQ, const M2LScaledArgs &a, const TM *Q, const TM *tin,
                       const double *logt, const TI *in, TO *out) {
    if (a.ncols <= 0) return;
    const unsigned blocks = (unsigned)((a.ncols + 15) / 16);
    switch (PQ) {
        case 16: launch_m2l_scaled<TI, TO, TM, 1>(s, nw, blocks, a, Q, tin, logt, in, out); break;
        case 32: launch_m2l_scaled<TI, TO, TM, 2>(s, nw, blocks, a, Q, tin, logt, in, out); break;
        case 48: launch_m2l_scaled<TI, TO, TM, 3>(s, nw, blocks, a, Q, tin, logt, in, out); break;
        case 64: launch_m2l_scaled<TI, TO, TM, 4>(s, nw, blocks, a, Q, tin, logt, in, out); break;
        default: throw Error(VP_EUNSUPPORTED, "unsupported expansion size");
    }
    VP_LAUNCH_CHECK();
}

static TranslateArgs expansion_args(vp_plan_s *P, const int32_t *cols, int nboxes, const int32_t *slots, int nops,
                                    int logrow) {
    TranslateArgs a;
    a.cols_box = cols;
    a.ncols = nboxes * P->nbatch;
    a.nbatch = P->nbatch;
    a.slots = slots;
    a.nops = nops;
    a.in = ColAddr{P->PD, (int64_t)P->nbatch * P->PD, nullptr};
    a.out = a.in;
    a.nrows_out = P->PD;
    a.logrow = logrow;
    a.level = P->tree.level;
    a.logside = P->tree.d_logside;
    a.zero_col = P->zero_col;
    return a;
}

// ----------------------------------------------------------------------------
// Host orchestration of one evaluation
// ----------------------------------------------------------------------------
static PointRoles roles(vp_plan_s *P, bool adjoint) {
    Tree &T = P->tree;
    PointRoles R;
    if (!adjoint) {
        R = {P->sx, P->sy, T.sb, T.se, P->tx, P->ty, T.tb, T.te, P->n, P->m};
    } else {
        R = {P->tx, P->ty, T.tb, T.te, P->sx, P->sy, T.sb, T.se, P->m, P->n};
    }
    return R;
}

static BoxGeo geo(vp_plan_s *P) {
    Tree &T = P->tree;
    return BoxGeo{T.level, T.ix, T.iy, T.parent, T.child, T.nchild, T.cx, T.cy, T.d_side, T.d_logside};
}

// Oversampled boxes (Section 4.2, eq. fk_basis / eq. Tnm, upsampled as in
// Section 3.2): the charge of source j = out_start[b] + r is
// w_j (O f_b)_r, O the q^2 x p^2 tensor-product Chebyshev map, written
// straight into sorted order.  One workgroup per box; the box's p^2 density
// values of one density at a time in LDS, threads over the q^2 rows (O^T
// read with the threads along a row of O^T: coalesced).
__global__ void k_interp_charge(const int64_t *__restrict__ in_start, const int64_t *__restrict__ out_start,
                                int p2, int q2, const double *__restrict__ OT, const double *__restrict__ f,
                                int64_t nd, const int32_t *__restrict__ sinv, const double *__restrict__ w,
                                int nbatch, int64_t n, double *__restrict__ q) {
    __shared__ double sf[1024];
    const int64_t b = blockIdx.x;
    const int64_t i0 = in_start[b], j0 = out_start[b];
    for (int bt = 0; bt < nbatch; ++bt) {
        for (int k = threadIdx.x; k < p2; k += blockDim.x) sf[k] = f[(int64_t)bt * nd + i0 + k];
        __syncthreads();
        for (int r = threadIdx.x; r < q2; r += blockDim.x) {
            double acc = 0.0;
            for (int k = 0; k < p2; ++k) acc = fma(OT[(int64_t)k * q2 + r], sf[k], acc);
            const int64_t j = j0 + r;
            q[(int64_t)bt * n + sinv[j]] = w[j] * acc;
        }
        __syncthreads();
    }
}

// The adjoint's finish on an oversampled plan: out[b][i0 + k] +=
// sum_r O[r][k] w_j acc[b][sinv[j]] (j = out_start + r): O^T applied to the
// weighted FMM sums at the box's sources, added to the transposed correction.
__global__ void k_interp_adjoint(const int64_t *__restrict__ in_start, const int64_t *__restrict__ out_start,
                                 int p2, int q2, const double *__restrict__ O, const double *__restrict__ acc,
                                 const double *__restrict__ acc2, int64_t n, const int32_t *__restrict__ sinv,
                                 const double *__restrict__ w, int nbatch, int64_t nd, double *__restrict__ out) {
    __shared__ double sv[1024];
    const int64_t b = blockIdx.x;
    const int64_t i0 = in_start[b], j0 = out_start[b];
    for (int bt = 0; bt < nbatch; ++bt) {
        for (int r = threadIdx.x; r < q2; r += blockDim.x) {
            const int64_t j = j0 + r, k = (int64_t)bt * n + sinv[j];
            sv[r] = w[j] * (acc2 ? acc[k] + acc2[k] : acc[k]);
        }
        __syncthreads();
        for (int c = threadIdx.x; c < p2; c += blockDim.x) {
            double s = 0.0;
            for (int r = 0; r < q2; ++r) s = fma(O[(int64_t)r * p2 + c], sv[r], s);
            double *o = out + (int64_t)bt * nd + i0 + c;
            *o = s + *o;
        }
        __syncthreads();
    }
}

void prepare_charges(vp_plan_s *P, const double *f, bool adjoint, bool grad) {
    int64_t len = adjoint ? P->m : P->n;
    const int32_t *perm = adjoint ? P->tperm : P->sperm;
    const double *w = adjoint ? nullptr : P->sw;
    P->q_valid = true;
    if (!adjoint && P->os_p > 0) {
        P->qi_valid = false;
        P->stage_begin(VP_STAGE_CHARGE);
        hipLaunchKernelGGL(k_interp_charge, dim3((unsigned)P->os_nbox), dim3(256), 0, P->stream, P->os_in, P->os_out,
                           P->os_p * P->os_p, P->os_q * P->os_q, P->os_OT, f, P->nd, P->sinv, P->w_user,
                           P->nbatch, P->n, P->q);
        VP_LAUNCH_CHECK();
        P->stage_end(VP_STAGE_CHARGE);
        return;
    }
    P->stage_begin(VP_STAGE_CHARGE);
    // the density-fastest copy only for the one-wave near-table kernel, its one reader
    // (the table kernel addresses it by 32-bit byte offsets and 24-bit point indices)
    P->qi_valid = P->qi != nullptr && P->table_nw == 1 &&
                  (P->qi_zero + QI_ZERO_PTS) * P->nbatch * 8 < ((int64_t)1 << 32) &&
                  P->qi_zero + QI_ZERO_PTS < (1 << 24);
    P->q_valid = !(P->qi_valid && P->q_pattern_only && !adjoint && !grad);
    // the leaf P2M fused into the charge pass: every leaf a pattern leaf of 64
    // nodes whose multipoles the fixed-matrix P2M forms (16 densities)
    const NearTables &N = P->near;
    const int rb = P->PD / 16;
    P->p2m_in_charges = !P->q_valid && P->nbatch == 16 && P->tree.nlevels >= 3 && N.active && N.npat == 64 &&
                        P->PD % 16 == 0 && rb >= 1 && rb <= 4 && N.n_p2m_leaf_cols == P->tree.nleaf &&
                        (P->fp32 ? N.p2m_op_f32 != nullptr : N.p2m_op != nullptr);
    if (P->p2m_in_charges) {
        const int nl = N.n_p2m_leaf_cols;
        // two workgroups per compute unit (the register budget), each looping over leaves
        const unsigned grid = (unsigned)std::min((nl + 3) / 4, 512);
        switch (rb * 2 + (P->fp32 ? 1 : 0)) {
#define VP_P2MQ(RB)                                                                                              \
    case RB * 2:                                                                                                 \
        hipLaunchKernelGGL((k_p2m_charge<double, RB, 16>), dim3(grid), dim3(256), 0, P->stream, N.p2m_cols, nl,  \
                           P->tree.sb, perm, w, f, len, N.p2m_op, P->qi, static_cast<double *>(P->Mexp), P->PD); \
        break;                                                                                                   \
    case RB * 2 + 1:                                                                                             \
        hipLaunchKernelGGL((k_p2m_charge<float, RB, 16>), dim3(grid), dim3(256), 0, P->stream, N.p2m_cols, nl,   \
                           P->tree.sb, perm, w, f, len, N.p2m_op_f32, P->qi, static_cast<float *>(P->Mexp),      \
                           P->PD);                                                                               \
        break;
            VP_P2MQ(1) VP_P2MQ(2) VP_P2MQ(3) VP_P2MQ(4)
#undef VP_P2MQ
        }
    } else if (P->qi_valid)
        hipLaunchKernelGGL(k_charge_il, dim3((unsigned)((len + 63) / 64)), dim3(64),
                           64 * (P->nbatch + 1) * sizeof(double), P->stream, f, perm, w,
                           P->q_valid ? P->q : nullptr, len, P->nbatch, P->qi);
    else
        hipLaunchKernelGGL(k_charge, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, P->stream, f, perm, w,
                           P->q, len, P->nbatch);
    VP_LAUNCH_CHECK();
    P->stage_end(VP_STAGE_CHARGE);
}

// fixed-matrix launches on pattern leaves (launch_pattern_ops)
enum { PAT_P2M = 0, PAT_L2P = 1 };
template <class E>
static void run_pattern_op(vp_plan_s *P, const PointRoles &R, int kind, double *acc = nullptr,
                           FinishArgs fin = FinishArgs());

// M2L of the V lists (and X-list virtual children) of one level range
// (part 0: levels from the split level on, part 1: the levels below) in one
// launch, by the plan's M2L mode
template <class E>
static void launch_m2l(vp_plan_s *P, int part) {
    Tree &T = P->tree;
    const M2LSched &S = P->m2l[part];
    if (S.nboxes == 0) return;
    hipStream_t s = P->stream;
    const int nb = P->nbatch, Pn = P->P, PD = P->PD;
    E *M = static_cast<E *>(P->Mexp);
    E *L = static_cast<E *>(P->Lexp);
    const bool f32 = sizeof(E) == 4;
    const Operators &O = P->ops;
    TranslateArgs a = expansion_args(P, S.cols, S.nboxes, T.v_slot, NOFF, 2 * Pn);
    a.tile_ptr = S.tptr;
    a.tile_ops = S.tops;
    a.tile_order = S.torder;
    a.xinit = P->x_init;
    if (P->m2l_mode == VP_M2L_FP64_SCALED || P->m2l_mode == VP_M2L_FP32_SCALED) {
        M2LScaledArgs sa;
        sa.cols_box = S.cols;
        sa.ncols = a.ncols;
        sa.nbatch = nb;
        sa.tile_ptr = S.tptr;
        sa.tile_ops = S.tops;
        sa.tile_src = S.tsrc;
        // the launch below the split level has few tiles on small trees: give
        // each tile the most waves there (its latency sets the coarse chain);
        // the one-wave form addresses the multipoles by 32-bit offsets
        const int64_t mbytes = P->mexp_boxes() * nb * PD * (int64_t)sizeof(E);
        const bool wave_fits = mbytes < ((int64_t)1 << 32) && P->zero_box() < (1 << 24);
        int nw = part == 1 && (a.ncols + 15) / 16 < 1024 ? 4 : P->m2l_nw;
        if (nw == 1 && !wave_fits) nw = 2;
        sa.zero_box = (int)P->zero_box();
        sa.tile_order = nw == 1 ? S.torder4 : S.torder;
        sa.P = Pn;
        sa.box_stride = (int64_t)nb * PD;
        sa.bt_stride = PD;
        sa.PD = PD;
        sa.zero_col = P->zero_col;
        sa.xinit = P->x_init;
        sa.level = T.level;
        sa.logside = T.d_logside;
        if (!f32)
            m2l_scaled<double, double, double>(s, nw, O.PQ, sa, O.m2l_q64, O.m2l_tin64, O.m2l_logt,
                                               (const double *)M, (double *)L);
        else if (P->m2l_mode == VP_M2L_FP32_SCALED)
            m2l_scaled<float, float, float>(s, nw, O.PQ, sa, O.m2l_q32, O.m2l_tin32, O.m2l_logt,
                                            (const float *)M, (float *)L);
        else
            m2l_scaled<float, float, double>(s, nw, O.PQ, sa, O.m2l_q64, O.m2l_tin64, O.m2l_logt,
                                             (const float *)M, (float *)L);
    } else if (!f32) {
        translate_m2l<double, double, double, false>(s, P->m2l_nw, PD, a, P->ops.m2l_f64, nullptr,
                                                     (const double *)M, (double *)L);
    } else if (P->m2l_mode == VP_M2L_FP32_SPLIT) {
        translate_m2l<float, float, float, true>(s, P->m2l_nw, PD, a, P->ops.m2l_f32, P->ops.m2l_f32_lo,
                                                 (const float *)M, (float *)L);
    } else if (P->m2l_mode == VP_M2L_FP64_MFMA) {
        translate_m2l<float, float, double, false>(s, P->m2l_nw, PD, a, P->ops.m2l_f64, nullptr,
                                                   (const float *)M, (float *)L);
    } else {
        translate_m2l<float, float, float, false>(s, P->m2l_nw, PD, a, P->ops.m2l_f32, nullptr,
                                                  (const float *)M, (float *)L);
    }
}

// Leaf multipoles on the VALU: every leaf and virtual child of an X-list
// source, or with tables only those the fixed matrices do not serve
template <class E>
static void run_p2m(vp_plan_s *P, const PointRoles &R, const BoxGeo &G, bool tables) {
    Tree &T = P->tree;
    const int nb = P->nbatch, Pn = P->P, PD = P->PD;
    const bool f32 = sizeof(E) == 4;
    const E *invk = f32 ? (const E *)P->ops.inv_k_f32 : (const E *)P->ops.inv_k;
    const size_t lds = sizeof(E) * 2 * 16 * Pn;
    const P2MJob *jobs = tables ? P->near.p2m_jobs_rest : (R.sb == T.sb ? P->p2m_jobs : P->p2m_jobs_t);
    const int njobs = tables ? P->near.n_p2m_jobs_rest : P->n_p2m_jobs;
    if (njobs <= 0) return;
    hipLaunchKernelGGL(k_p2m<E>, dim3(njobs), dim3(64), lds, P->stream, R, jobs, P->q, nb, Pn, PD, invk,
                       static_cast<E *>(P->Mexp));
    VP_LAUNCH_CHECK();
}

// Densities per workgroup of a per-level M2M / L2L launch: all of them when
// the level has enough boxes to fill the chip, else fewer, with the
// densities spread over blockIdx.y (a wave otherwise walks every density of
// its boxes in turn, and the coarse levels' few waves set the launch time)
static int density_chunk(int nblocks, int nbatch) {
    const int want = std::max(1, std::min(nbatch, 2048 / std::max(nblocks, 1)));
    return (nbatch + want - 1) / want;
}

// M2M for the parents on levels l_hi down to l_lo (one launch per level)
template <class E>
static void run_m2m(vp_plan_s *P, const BoxGeo &G, int l_hi, int l_lo) {
    hipStream_t s = P->stream;
    const int nb = P->nbatch, Pn = P->P, PD = P->PD;
    E *M = static_cast<E *>(P->Mexp);
    const bool f32 = sizeof(E) == 4;
    const Operators &O = P->ops;
    const E *shq = f32 ? (const E *)O.sh_qt32[0] : (const E *)O.sh_qt64[0];
    const E *shi = f32 ? (const E *)O.sh_tin32[0] : (const E *)O.sh_tin64[0];
    const E *sho = f32 ? (const E *)O.sh_tout32[0] : (const E *)O.sh_tout64[0];
    for (int l = l_hi; l >= l_lo; --l) {
        const int c0 = P->m2m_begin[l], c1 = P->m2m_begin[l + 1];
        if (c1 <= c0) continue;
        if (!f32 && nb % 16 == 0 && (O.PR == 16 || O.PR == 32)) {
            // one parent's sixteen densities per wave on the matrix cores
            const int ntile = (c1 - c0) * (nb / 16);
            const dim3 grid((unsigned)((ntile + 3) / 4));
            const int4 *cs = reinterpret_cast<const int4 *>(P->m2m_cslot) + c0;
            if (O.PR == 16)
                hipLaunchKernelGGL((k_m2m_wave<1>), grid, dim3(256), 0, s, P->m2m_parents + c0, cs, c1 - c0, nb, Pn,
                                   PD, O.PR, (int)P->zero_box(), (const double *)shq, (const double *)shi, (const double *)sho,
                                   (double *)M);
            else
                hipLaunchKernelGGL((k_m2m_wave<2>), grid, dim3(256), 0, s, P->m2m_parents + c0, cs, c1 - c0, nb, Pn,
                                   PD, O.PR, (int)P->zero_box(), (const double *)shq, (const double *)shi, (const double *)sho,
                                   (double *)M);
            VP_LAUNCH_CHECK();
            continue;
        }
        const int chunk = density_chunk(c1 - c0, nb);
        const dim3 grid((unsigned)(c1 - c0), (unsigned)((nb + chunk - 1) / chunk));
        switch (O.PR) {
#define VP_M2M(PR)                                                                                                 \
    case PR:                                                                                                       \
        hipLaunchKernelGGL((k_m2m<E, PR>), grid, dim3(64), 0, s, P->m2m_parents + c0,                            \
                           reinterpret_cast<const int4 *>(P->m2m_cslot) + c0, nb, Pn, PD, shq, shi, sho, M, chunk); \
        break;
            VP_M2M(16) VP_M2M(32) VP_M2M(64)
#undef VP_M2M
            default: throw Error(VP_EUNSUPPORTED, "unsupported expansion size");
        }
        VP_LAUNCH_CHECK();
    }
}

// L2L into the boxes of levels l_lo .. l_hi (one launch per level)
template <class E>
static void run_l2l(vp_plan_s *P, const BoxGeo &G, int l_lo, int l_hi) {
    hipStream_t s = P->stream;
    const int nb = P->nbatch, Pn = P->P, PD = P->PD;
    E *L = static_cast<E *>(P->Lexp);
    const bool f32 = sizeof(E) == 4;
    const Operators &O = P->ops;
    const E *shq = f32 ? (const E *)O.sh_qt32[1] : (const E *)O.sh_qt64[1];
    const E *shi = f32 ? (const E *)O.sh_tin32[1] : (const E *)O.sh_tin64[1];
    const E *sho = f32 ? (const E *)O.sh_tout32[1] : (const E *)O.sh_tout64[1];
    for (int l = std::max(l_lo, 3); l <= l_hi; ++l) {
        const int c0 = P->lvl_box_begin[l], c1 = P->lvl_box_begin[l + 1];
        if (c1 <= c0) continue;
        const unsigned nblk = (unsigned)((c1 - c0 + 64 / O.PR - 1) / (64 / O.PR));
        const int chunk = density_chunk((int)nblk, nb);
        const dim3 grid(nblk, (unsigned)((nb + chunk - 1) / chunk));
        switch (O.PR) {
#define VP_L2L(PR)                                                                                               \
    case PR:                                                                                                     \
        hipLaunchKernelGGL((k_l2l<E, PR>), grid, dim3(64), 0, s, P->lvl_boxes + c0, P->lvl_pcls + c0,           \
                           c1 - c0, nb, Pn, PD, shq, shi, sho, L, chunk);                                        \
        break;
            VP_L2L(16) VP_L2L(32) VP_L2L(64)
#undef VP_L2L
            default: throw Error(VP_EUNSUPPORTED, "unsupported expansion size");
        }
        VP_LAUNCH_CHECK();
    }
}

// P2L of the X-list entries two or more levels apart (writes those boxes'
// local expansions before M2L adds to them)
template <class E>
static void run_p2l(vp_plan_s *P, const PointRoles &R, const BoxGeo &G) {
    if (P->n_x_boxes <= 0) return;
    const int Pn = P->P;
    const bool f32 = sizeof(E) == 4;
    const E *invk = f32 ? (const E *)P->ops.inv_k_f32 : (const E *)P->ops.inv_k;
    const size_t lds = sizeof(E) * 2 * 16 * Pn;
    hipLaunchKernelGGL(k_p2l<E>, dim3(P->n_x_boxes), dim3(64), lds, P->stream, R, G, P->x_boxes, P->xr_ptr,
                       P->xr_idx, P->q, P->nbatch, Pn, P->PD, invk, static_cast<E *>(P->Lexp));
    VP_LAUNCH_CHECK();
}

template <int NB, bool GRAD, bool ACCUM>
static void launch_p2p(vp_plan_s *P, const PointRoles &R, const int32_t *leaves, int nleaves, const int32_t *uptr,
                       const int32_t *uidx, const P2PGather *gs, int bt0, double *acc) {
    if (nleaves <= 0) return;
    const double2 *lt = (const double2 *)P->ops.log_table;
    if (gs && gs->ptr)
        hipLaunchKernelGGL((k_p2p<NB, GRAD, ACCUM, true>), dim3(nleaves), dim3(64), 0, P->stream, R, leaves, uptr,
                           uidx, *gs, P->q, P->nbatch, bt0, lt, acc);
    else
        hipLaunchKernelGGL((k_p2p<NB, GRAD, ACCUM, false>), dim3(nleaves), dim3(64), 0, P->stream, R, leaves, uptr,
                           uidx, P2PGather(), P->q, P->nbatch, bt0, lt, acc);
    VP_LAUNCH_CHECK();
}

// Pairwise near field over (leaves, U lists); densities in groups of 16/8/4/2/1.
template <bool GRAD, bool ACCUM>
static void run_p2p(vp_plan_s *P, const PointRoles &R, const int32_t *leaves, int nleaves, const int32_t *uptr,
                    const int32_t *uidx, const P2PGather *gs, double *acc) {
    int nb = P->nbatch;
    for (int bt0 = 0; bt0 < nb;) {
        const int left = nb - bt0;
        if (left >= 16) {
            launch_p2p<16, GRAD, ACCUM>(P, R, leaves, nleaves, uptr, uidx, gs, bt0, acc);
            bt0 += 16;
        } else if (left >= 8) {
            launch_p2p<8, GRAD, ACCUM>(P, R, leaves, nleaves, uptr, uidx, gs, bt0, acc);
            bt0 += 8;
        } else if (left >= 4) {
            launch_p2p<4, GRAD, ACCUM>(P, R, leaves, nleaves, uptr, uidx, gs, bt0, acc);
            bt0 += 4;
        } else if (left >= 2) {
            launch_p2p<2, GRAD, ACCUM>(P, R, leaves, nleaves, uptr, uidx, gs, bt0, acc);
            bt0 += 2;
        } else {
            launch_p2p<1, GRAD, ACCUM>(P, R, leaves, nleaves, uptr, uidx, gs, bt0, acc);
            bt0 += 1;
        }
    }
}

// Near-field tables of congruent leaves: acc[:, leaf] += sum_o K_{l,o} q[:, nbr_o(leaf)],
// all table levels in one launch (operator index = level block * NTOPS + slot).
template <int RB>
static void launch_tables(vp_plan_s *P, const PointRoles &R, const double *K) {
    NearTables &N = P->near;
    constexpr int S = RB * 4;
    TranslateArgs a;
    a.cols_box = N.tab_cols;
    a.ncols = N.tab_cols_begin.back() * P->nbatch;
    a.nbatch = P->nbatch;
    a.slots = N.tab_slot;
    a.nops = NTOPS * (int)N.tab_levels.size();
    a.tile_ptr = N.tile_ptr;
    a.tile_ops = N.tile_ops;
    a.tile_order = N.tile_order;
    a.in = ColAddr{R.nsrc, 0, R.sb};
    a.out = ColAddr{R.ntgt, 0, R.tb};
    a.nrows_out = N.npat;
    a.logrow = -1;
    a.level = P->tree.level;
    a.logside = P->tree.d_logside;
    a.zero_col = P->zero_col;
    if (a.ncols <= 0) return;
    // every table leaf's sums are stored by its one tile (the other leaves are zeroed)
    const unsigned blocks = (unsigned)((a.ncols + 15) / 16);
    bool done = false;
    if constexpr (RB <= 4) {
        // one wave over two tiles (larger patterns would spill: the two-wave form serves them)
        if (P->table_nw == 1) {
            a.tile_ptr = N.tile2_ptr;
            a.tile_ops = N.tile2_ops;
            a.tile_order = N.tile2_order;
            const dim3 grid((unsigned)((a.ncols + 31) / 32));
            a.in_zero = (int)P->qi_zero;
            if (P->qi_valid && P->nbatch == 16)
                hipLaunchKernelGGL((k_tables_ct<RB, S, 2, true, 16>), grid, dim3(64), 0, P->stream, a, K, P->qi,
                                   P->acc);
            else if (P->qi_valid)
                hipLaunchKernelGGL((k_tables_ct<RB, S, 2, true>), grid, dim3(64), 0, P->stream, a, K, P->qi,
                                   P->acc);
            else
                hipLaunchKernelGGL((k_tables_ct<RB, S, 2, false>), grid, dim3(64), 0, P->stream, a, K, P->q,
                                   P->acc);
            done = true;
        }
    }
    if (done) {
    } else if (P->table_nw <= 2)
        hipLaunchKernelGGL((k_translate_split<double, double, double, RB, S, false, false, 2>), dim3(blocks),
                           dim3(128), 0, P->stream, a, K, (const double *)nullptr, P->q, P->acc);
    else
        hipLaunchKernelGGL((k_translate_split<double, double, double, RB, S, false, false, 4>), dim3(blocks),
                           dim3(256), 0, P->stream, a, K, (const double *)nullptr, P->q, P->acc);
    VP_LAUNCH_CHECK();
}

static void run_tables(vp_plan_s *P, const PointRoles &R, const double *K) {
    switch (P->near.npat) {
        case 16: launch_tables<1>(P, R, K); break;
        case 32: launch_tables<2>(P, R, K); break;
        case 48: launch_tables<3>(P, R, K); break;
        case 64: launch_tables<4>(P, R, K); break;
        case 80: launch_tables<5>(P, R, K); break;
        case 96: launch_tables<6>(P, R, K); break;
        case 112: launch_tables<7>(P, R, K); break;
        case 128: launch_tables<8>(P, R, K); break;
        default: throw Error(VP_EINTERNAL, "unsupported pattern size");
    }
}

// One fixed operator over ncols columns (k_fixed_apply): four waves per
// workgroup, at most four resident workgroups per compute unit's worth of
// tiles (the kernel walks the rest with a grid stride).
template <class TI, class TO, class TM, int RB, int S, bool ACCUM, bool FIN = false>
static void launch_fixed_apply(vp_plan_s *P, const int32_t *cols_box, int ncols, ColAddr ia, ColAddr oa,
                               int nrows_out, const TM *A, const TI *in, TO *out, const int32_t *addflag = nullptr,
                               FinishArgs fin = FinishArgs()) {
    if (ncols <= 0) return;
    const int ntiles = (ncols + 15) / 16;
    // the operator in LDS when it fits in 32 KB (up to five workgroups per
    // compute unit), else in registers
    constexpr bool ALDS = (size_t)RB * S * 64 * sizeof(TM) <= 32768;
    const unsigned grid = (unsigned)std::min((ntiles + 3) / 4, ALDS ? 1280 : 512);
    hipLaunchKernelGGL((k_fixed_apply<TI, TO, TM, RB, S, ACCUM, FIN, ALDS>), dim3(grid), dim3(256), 0, P->stream,
                       cols_box, ncols, P->nbatch, ia, oa, nrows_out, A, in, out, addflag, fin);
    VP_LAUNCH_CHECK();
}

// zero the sums of the targets of the listed leaves (all densities)
__global__ void k_zero_leaves(const int32_t *__restrict__ leaves, const int32_t *__restrict__ tb,
                              const int32_t *__restrict__ te, int nbatch, int64_t ntgt, double *__restrict__ acc) {
    const int b = leaves[blockIdx.x];
    const int t0 = tb[b], nt = te[b] - t0;
    for (int e = threadIdx.x; e < nt * nbatch; e += blockDim.x)
        acc[(int64_t)(e / nt) * ntgt + t0 + e % nt] = 0.0;
}

static void zero_leaves(vp_plan_s *P, const PointRoles &R, const int32_t *leaves, int n, double *acc) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero_leaves, dim3(n), dim3(256), 0, P->stream, leaves, R.tb, R.te, P->nbatch, R.ntgt, acc);
    VP_LAUNCH_CHECK();
}

// Fixed-matrix launches on pattern leaves: P2M (q -> M, with the quadrant
// P2M of pattern X-list sources into their virtual-child columns) and L2P
// (L -> acc)
template <class E, int RBP, int RBE>
static void launch_pattern_ops(vp_plan_s *P, const PointRoles &R, int kind, double *acc, FinishArgs fin) {
    NearTables &N = P->near;
    const bool f32 = sizeof(E) == 4;
    TranslateArgs a;
    a.nbatch = P->nbatch;
    a.slots = N.ident_slot;
    a.nops = 1;
    a.logrow = -1;
    a.level = P->tree.level;
    a.logside = P->tree.d_logside;
    a.zero_col = P->zero_col;
    if (kind == PAT_P2M) {
        // rows = expansion (RBE blocks), cols = pattern points (RBP*16); operator
        // 0 for pattern leaves, 1 + quadrant for the virtual children of pattern
        // X-list sources (zero outside the quadrant's points); the columns are
        // grouped by operator, so a 64-column block uses one (two at a boundary).
        // This launch runs beside the VALU P2M and the correction at the start
        // of an evaluation: the four-column-tile form (fewer waves) suits it.
        constexpr int RB = RBE, S = RBP * 4;
        constexpr bool LDSA = translate_ldsa<E, RB, S, false>();
        constexpr size_t lds = LDSA ? translate_lds_bytes<E, RB, S, false>() : 0;
        a.in = ColAddr{R.nsrc, 0, R.sb};
        a.out = ColAddr{P->PD, (int64_t)P->nbatch * P->PD, nullptr};
        a.nrows_out = P->PD;
        const E *op = f32 ? (const E *)N.p2m_op_f32 : (const E *)N.p2m_op;
        // the leading pattern-leaf columns all use operator 0: one fixed operator
        const int n0 = N.n_p2m_leaf_cols;
        if (n0 > 0 && P->q_valid)
            launch_fixed_apply<double, E, E, RB, S, false>(P, N.p2m_cols, n0 * P->nbatch, a.in, a.out, a.nrows_out,
                                                           op, P->q, static_cast<E *>(P->Mexp));
        else if (n0 > 0) {
            // from the density-fastest copy: point k of column (box, d) at (start + k) nbatch + d
            const ColAddr il{1, 0, R.sb, P->nbatch, P->nbatch};
            launch_fixed_apply<double, E, E, RB, S, false>(P, N.p2m_cols, n0 * P->nbatch, il, a.out, a.nrows_out,
                                                           op, P->qi, static_cast<E *>(P->Mexp));
        }
        // the quadrant columns of X-list sources (operators 1..4)
        a.cols_box = N.p2m_cols + n0;
        a.ncols = (N.n_p2m_cols - n0) * P->nbatch;
        a.slots = N.p2m_slot;
        a.nops = 5;
        if (a.ncols <= 0) return;
        hipLaunchKernelGGL((k_translate<double, E, E, RB, S, false, false, LDSA>),
                           dim3((unsigned)((a.ncols + 63) / 64)), dim3(256), lds, P->stream, a, op, (const E *)nullptr,
                           P->q, static_cast<E *>(P->Mexp));
    } else {
        // rows = pattern points (RBP blocks, one per wave), cols = expansions
        a.cols_box = N.l2p_pat;
        a.ncols = N.n_l2p_pat * P->nbatch;
        a.in = ColAddr{P->PD, (int64_t)P->nbatch * P->PD, nullptr};
        a.out = ColAddr{R.ntgt, 0, R.tb};
        a.nrows_out = N.npat;
        if (a.ncols <= 0) return;
        const E *op = f32 ? (const E *)N.l2p_op_f32 : (const E *)N.l2p_op;
        if constexpr (sizeof(E) == 8) {
            if (fin.u && N.par_l2p) {
                // the deepest level from the leaves' and their parents' local expansions
                L2PFinArgs fa;
                fa.rec = N.l2p_rec;
                int maxq = 0;
                for (int q = 0; q < 5; ++q) fa.qbeg[q] = N.l2p_qbeg[q];
                for (int q = 0; q < 4; ++q) maxq = std::max(maxq, N.l2p_qbeg[q + 1] - N.l2p_qbeg[q]);
                fa.box_stride = (int64_t)P->nbatch * P->PD;
                fa.PD = P->PD;
                fa.tb = R.tb;
                fa.near = fin.near;
                fa.ntgt = R.ntgt;
                fa.perm = fin.perm;
                fa.u = fin.u;
                fa.m = fin.m;
                // two workgroups per compute unit (64 KB of operators each), a
                // quarter of them per class, in groups of 32 (the kernel's
                // class-to-XCD mapping)
                const unsigned grid = 32u * (unsigned)std::max(1, std::min(16, (maxq + 127) / 128));
                if (N.npat != RBP * 16) throw Error(VP_EINTERNAL, "pattern size off its row blocks");
                if (fin.add_u)
                    hipLaunchKernelGGL((k_l2p_fin<RBP, RBE * 4, true>), dim3(grid), dim3(256), 0, P->stream, fa,
                                       N.l2p_km, N.par_km, static_cast<const double *>(P->Lexp));
                else
                    hipLaunchKernelGGL((k_l2p_fin<RBP, RBE * 4, false>), dim3(grid), dim3(256), 0, P->stream, fa,
                                       N.l2p_km, N.par_km, static_cast<const double *>(P->Lexp));
                VP_LAUNCH_CHECK();
                return;
            }
        }
        if (fin.u)
            launch_fixed_apply<E, double, E, RBP, RBE * 4, false, true>(
                P, a.cols_box, a.ncols, a.in, a.out, a.nrows_out, op, static_cast<const E *>(P->Lexp), acc,
                nullptr, fin);
        else
            launch_fixed_apply<E, double, E, RBP, RBE * 4, false>(P, a.cols_box, a.ncols, a.in, a.out, a.nrows_out,
                                                                 op, static_cast<const E *>(P->Lexp), acc,
                                                                 N.far_add);
        return;
    }
    VP_LAUNCH_CHECK();
}

bool pattern_op_supported(int npat, int PD) {
    return (npat == 16 || npat == 32 || npat == 64) && PD >= 16 && PD <= 64 && PD % 16 == 0;
}

template <class E>
static void run_pattern_op(vp_plan_s *P, const PointRoles &R, int kind, double *acc, FinishArgs fin) {
    const int key = P->near.npat / 16 * 16 + P->PD / 16;
    switch (key) {
#define VP_PAT(NP, NE) \
    case NP * 16 + NE: launch_pattern_ops<E, NP, NE>(P, R, kind, acc, fin); break;
        VP_PAT(1, 1) VP_PAT(1, 2) VP_PAT(1, 3) VP_PAT(1, 4)
        VP_PAT(2, 1) VP_PAT(2, 2) VP_PAT(2, 3) VP_PAT(2, 4)
        VP_PAT(4, 1) VP_PAT(4, 2) VP_PAT(4, 3) VP_PAT(4, 4)
#undef VP_PAT
        default: throw Error(VP_EUNSUPPORTED, "pattern/order combination without a pattern operator");
    }
}

template <class E, bool GRAD>
static void run_far(vp_plan_s *P, const PointRoles &R, const BoxGeo &G, double *acc, bool tables, int parts,
                    FinishArgs fin = FinishArgs()) {
    // parts: bit 0 the local expansions at the targets (L2P), bit 1 the W lists (M2P)
    Tree &T = P->tree;
    NearTables &N = P->near;
    auto far = [&](const int32_t *leaves, int nleaves, const int32_t *done, int pt) {
        if (nleaves <= 0) return;
        // four waves share a leaf's W list; local expansions alone take one wave
        const unsigned threads = pt == 1 ? 64 : 256;
        hipLaunchKernelGGL((k_far<E, GRAD>), dim3(nleaves), dim3(threads), 0, P->stream, R, G, leaves, T.lptr[2],
                           T.lidx[2], P->nbatch, P->P, P->PD, (const E *)P->Mexp, (const E *)P->Lexp, done, acc, pt);
        VP_LAUNCH_CHECK();
    };
    if (parts == 3) {
        // both in one launch per leaf
        if (tables) {
            run_pattern_op<E>(P, R, PAT_L2P, acc);
            far(N.far_leaves, N.n_far_leaves, N.local_done, 3);
        } else {
            far(T.leaves, T.nleaf, nullptr, 3);
        }
    } else if (parts == 1) {
        if (tables) {
            run_pattern_op<E>(P, R, PAT_L2P, acc, fin);
            far(N.l2p_rest, N.n_l2p_rest, nullptr, 1);
        } else {
            far(T.leaves, T.nleaf, nullptr, 1);
        }
    } else {
        far(P->w_leaves, P->n_w_leaves, nullptr, 2);
    }
}

static void correction_apply(vp_plan_s *P, const double *f, double *u, bool adjoint);
static void add_fmm_sums(vp_plan_s *P, double *u, bool adjoint);

// One evaluation on three streams (default priority; with VP_FLAG_ONE_STREAM
// everything runs on the plan's stream in the order written here):
//   third stream: VALU P2M, P2L | wait(upper) M2M of the levels below the
//                 split (then every multipole is done), their M2L and L2L
//   second stream: correction C f, near tables | wait(all multipoles) W lists
//                  at the targets (M2P), pairwise near field
//   plan's stream: fixed-matrix P2M | wait(VALU P2M) M2M from the finest
//                  level to the split level |
//                  wait(P2L) M2L of the levels from the split on | wait(coarse)
//                  L2L from the split level down | wait(second stream) local
//                  expansions at the targets, finish
// (the far field writes its own array; with gradients it runs whole on the
// plan's stream after the near field and adds to it)
template <class E>
static void run_passes(vp_plan_s *P, const PointRoles &R, const BoxGeo &G, bool adjoint, bool grad, const double *f,
                       double *u) {
    Tree &T = P->tree;
    NearTables &N = P->near;
    const bool tables = N.active && !grad;
    const bool one = P->one_stream;
    const bool fmm = T.nlevels >= 3;  // otherwise no box is well separated from another
    const int L0 = P->split_level, Lmax = T.nlevels - 1;
    const bool coarse = fmm && L0 > 2;
    // forward evaluation on an all-pattern grid: the L2P launch writes the output
    const bool fused = tables && fmm && N.fused_finish && !adjoint && u != nullptr;
    // and with the own-cell corrections folded into the near tables' self slot
    const bool folded = fused && N.corr_folded;
    hipStream_t ms = P->stream;
    hipStream_t s2 = one ? ms : P->aux, s3 = one ? ms : P->aux2;
    struct Restore {
        vp_plan_s *P;
        hipStream_t s;
        ~Restore() { P->stream = s; }
    } restore{P, ms};
    if (!one) {
        VP_HIP(hipEventRecord(P->ev_fork, ms));
        VP_HIP(hipStreamWaitEvent(s2, P->ev_fork, 0));
        VP_HIP(hipStreamWaitEvent(s3, P->ev_fork, 0));
    }
    // third stream: the VALU P2M first (the upward pass waits for it), P2L
    // (needs only the charges), then zero the far-field sums, which stay
    // apart from the near field so that the near field can run to the end of
    // the evaluation (ev_p2l covers the zeroing)
    P->stream = s3;
    if (fmm) {
        // VALU leaf multipoles (the fixed-matrix ones run on the plan's stream)
        P->stage_begin(VP_STAGE_P2M);
        run_p2m<E>(P, R, G, tables);
        P->stage_end(VP_STAGE_P2M);
        if (!one) VP_HIP(hipEventRecord(P->ev_p2m, s3));
        P->stage_begin(VP_STAGE_P2L);
        run_p2l<E>(P, R, G);
        P->stage_end(VP_STAGE_P2L);
    }
    if (tables) zero_leaves(P, R, N.zero_far, N.n_zero_far, P->acc_far);
    else if (!grad) fill_f64(P->acc_far, 0.0, (int64_t)P->nbatch * R.ntgt, P->stream);
    if (!one) VP_HIP(hipEventRecord(P->ev_p2l, s3));
    // second stream: correction (HBM bound) and the near field
    P->stream = s2;
    auto corr = [&] {
        if (u && !folded) correction_apply(P, f, u, adjoint);
    };
    auto tab = [&] {
        if (tables) {
            P->stage_begin(VP_STAGE_TABLES);
            run_tables(P, R, folded ? N.Kf : N.K);
            P->stage_end(VP_STAGE_TABLES);
        }
    };
    auto pair = [&] {
        P->stage_begin(VP_STAGE_P2P);
        if (grad) {
            run_p2p<true, false>(P, R, T.leaves, T.nleaf, T.lptr[0], T.lidx[0], nullptr, P->acc);
        } else if (tables) {
            run_p2p<false, true>(P, R, N.rest_leaves, N.n_rest_leaves, N.pair_uptr, N.pair_uidx, &N.g_rest,
                                 P->acc);
        } else {
            run_p2p<false, false>(P, R, T.leaves, T.nleaf, T.lptr[0], T.lidx[0],
                                  adjoint && !P->self ? &P->g_adj : &P->g_fwd, P->acc);
        }
        P->stage_end(VP_STAGE_P2P);
    };
    // with tables the table launch stores its leaves' sums; the other leaves
    // are zeroed for the pairwise kernel, which adds
    if (tables) zero_leaves(P, R, N.zero_near, N.n_zero_near, P->acc);
    corr();
    tab();
    // (the W lists and the pairwise near field follow once every multipole is done)
    // plan's stream: leaf multipoles and the upward pass down to the split level
    P->stream = ms;
    if (fmm) {
        if (tables && !P->p2m_in_charges) {
            P->stage_begin(VP_STAGE_P2M_PAT);
            run_pattern_op<E>(P, R, PAT_P2M);
            P->stage_end(VP_STAGE_P2M_PAT);
        }
        if (!one) VP_HIP(hipStreamWaitEvent(ms, P->ev_p2m, 0));
        P->stage_begin(VP_STAGE_M2M);
        run_m2m<E>(P, G, Lmax - 1, L0);
        P->stage_end(VP_STAGE_M2M);
    }
    // the W lists (M2P) need every multipole: after the upward pass; they go
    // on the third stream too (not with gradients, whose far field adds to the
    // near-field array)
    const bool w_apart = fmm && !grad;
    if (fmm && !one) VP_HIP(hipEventRecord(P->ev_upper, ms));
    if (coarse) {
        // the levels below the split, upward, M2L and downward; ev_m2p marks
        // every multipole done
        P->stream = s3;
        if (!one) VP_HIP(hipStreamWaitEvent(s3, P->ev_upper, 0));
        P->stage_begin(VP_STAGE_COARSE);
        run_m2m<E>(P, G, L0 - 1, 2);
        if (!one) VP_HIP(hipEventRecord(P->ev_m2p, s3));
        launch_m2l<E>(P, 1);
        run_l2l<E>(P, G, 3, L0 - 1);
        P->stage_end(VP_STAGE_COARSE);
        if (!one) VP_HIP(hipEventRecord(P->ev_coarse, s3));
        P->stream = ms;
    }
    // second stream: the W lists at the targets (far-field array) between the
    // near tables and the pairwise near field, once every multipole is done
    P->stream = s2;
    if (w_apart) {
        if (!one) {
            // every multipole (and, through the third stream, the zeroed far-field sums)
            if (coarse) {
                VP_HIP(hipStreamWaitEvent(s2, P->ev_m2p, 0));
            } else {
                VP_HIP(hipStreamWaitEvent(s2, P->ev_upper, 0));
                VP_HIP(hipStreamWaitEvent(s2, P->ev_p2l, 0));
            }
        }
        P->stage_begin(VP_STAGE_M2P);
        run_far<E, false>(P, R, G, P->acc_far, tables, 2);
        P->stage_end(VP_STAGE_M2P);
    }
    pair();
    P->stream = ms;
    if (fmm) {
        if (!one) VP_HIP(hipStreamWaitEvent(ms, P->ev_p2l, 0));
        P->stage_begin(VP_STAGE_M2L);
        launch_m2l<E>(P, 0);
        P->stage_end(VP_STAGE_M2L);
    } else if (!one) {
        VP_HIP(hipStreamWaitEvent(ms, P->ev_p2l, 0));  // join the third stream
    }
    // the second stream's end: the near field and the W lists
    if (!one) VP_HIP(hipEventRecord(P->ev_join, s2));
    if (fmm) {
        if (coarse && !one) VP_HIP(hipStreamWaitEvent(ms, P->ev_coarse, 0));
        P->stage_begin(VP_STAGE_L2L);
        // with the parents' L2P, the deepest level takes no L2L (forward only)
        run_l2l<E>(P, G, L0, fused && N.par_l2p ? N.par_level - 1 : Lmax);
        P->stage_end(VP_STAGE_L2L);
    }
    P->stage_begin(VP_STAGE_FAR);
    if (grad) {
        // the gradient sums go into the near-field array
        if (!one) VP_HIP(hipStreamWaitEvent(ms, P->ev_join, 0));
        if (fmm) run_far<E, true>(P, R, G, P->acc, false, 3);
    } else {
        // local expansions at the targets, after the W lists (same array, on
        // the second stream: the join covers them)
        if (!one) VP_HIP(hipStreamWaitEvent(ms, P->ev_join, 0));
        if (fused) {
            // the pattern L2P adds the near field and the correction row and
            // writes the output (the join also covers the correction)
            FinishArgs fin;
            fin.near = P->acc;
            fin.perm = P->tperm;
            fin.m = P->m;
            fin.u = u;
            fin.add_u = !folded;
            run_far<E, false>(P, R, G, P->acc_far, tables, 1, fin);
        } else if (fmm) {
            run_far<E, false>(P, R, G, P->acc_far, tables, 1);
        }
    }
    P->stage_end(VP_STAGE_FAR);
    if (u && !fused) add_fmm_sums(P, u, adjoint);
}

// one gather-GEMM launch over expansion columns (four operator slots per column)
template <int RB>
static void yk_translate(vp_plan_s *P, const TranslateArgs &a, const double *ops, const double *in, double *out,
                         bool accum) {
    constexpr int S = RB * 4;
    constexpr size_t lds = translate_lds_bytes<double, RB, S, false>();
    const unsigned grid = (unsigned)((a.ncols + 63) / 64);
    if (accum)
        hipLaunchKernelGGL((k_translate<double, double, double, RB, S, false, true, true>), dim3(grid), dim3(256), lds,
                           P->stream, a, ops, (const double *)nullptr, in, out);
    else
        hipLaunchKernelGGL((k_translate<double, double, double, RB, S, false, false, true>), dim3(grid), dim3(256),
                           lds, P->stream, a, ops, (const double *)nullptr, in, out);
    VP_LAUNCH_CHECK();
}

// Modified Helmholtz kernel on a uniform grid of congruent leaves: every
// stage a fixed matrix (vp_yukawa.hip), on the plan's stream in order --
// correction, near tables (store), pattern P2M, M2M per level upward, M2L
// of all levels in one launch (adding to zeroed locals), L2L per level
// downward (adding), pattern L2P (store), finish.  Targets are the nodes,
// so the adjoint is the same passes with the charges g and the weights
// applied at the finish.
static void run_yukawa(vp_plan_s *P, const PointRoles &R, bool adjoint, const double *f, double *u) {
    Tree &T = P->tree;
    NearTables &N = P->near;
    YukawaPlan &Y = P->yk;
    const int nb = P->nbatch, PD = P->PD, L = Y.leaf_level;
    double *M = static_cast<double *>(P->Mexp), *Lx = static_cast<double *>(P->Lexp);
    if (u) correction_apply(P, f, u, adjoint);
    P->stage_begin(VP_STAGE_TABLES);
    run_tables(P, R, N.K);
    P->stage_end(VP_STAGE_TABLES);
    const bool fmm = L >= 2;
    if (!fmm) {
        fill_f64(P->acc_far, 0.0, (int64_t)nb * R.ntgt, P->stream);
    } else {
        const ColAddr ex{PD, (int64_t)nb * PD, nullptr};
        auto gemm = [&](const int32_t *cols, int ncolbox, const int32_t *slots, const double *ops, const double *in,
                        double *out, bool accum) {
            if (ncolbox <= 0) return;
            TranslateArgs a;
            a.cols_box = cols;
            a.ncols = ncolbox * nb;
            a.nbatch = nb;
            a.slots = slots;
            a.nops = 4;
            a.in = ex;
            a.out = ex;
            a.nrows_out = PD;
            a.logrow = -1;
            a.level = T.level;
            a.logside = T.d_logside;
            a.zero_col = P->zero_col;
            switch (PD) {
                case 16: yk_translate<1>(P, a, ops, in, out, accum); break;
                case 32: yk_translate<2>(P, a, ops, in, out, accum); break;
                case 48: yk_translate<3>(P, a, ops, in, out, accum); break;
                case 64: yk_translate<4>(P, a, ops, in, out, accum); break;
                default: throw Error(VP_EUNSUPPORTED, "expansion size");
            }
        };
        const size_t AE = (size_t)PD * PD;
        // pattern P2M of the leaves (store)
        P->stage_begin(VP_STAGE_P2M_PAT);
        {
            const ColAddr pin{R.nsrc, 0, R.sb};
            switch (PD) {
#define VP_YP(RB)                                                                                                  \
    case RB * 16:                                                                                                  \
        launch_fixed_apply<double, double, double, RB, 16, false>(P, N.l2p_pat, N.n_l2p_pat * nb, pin, ex, PD, Y.p2m, \
                                                                  P->q, M);                                        \
        break;
                VP_YP(1) VP_YP(2) VP_YP(3) VP_YP(4)
#undef VP_YP
            }
        }
        P->stage_end(VP_STAGE_P2M_PAT);
        // M2M, finest parents first (store into the parents)
        P->stage_begin(VP_STAGE_M2M);
        for (int l = L - 1; l >= 2; --l)
            gemm(Y.d_parents[l], (int)Y.parents[l].size(), Y.cslot, Y.m2m + (size_t)l * 4 * AE, M, M, false);
        P->stage_end(VP_STAGE_M2M);
        // M2L of every level into zeroed locals
        P->stage_begin(VP_STAGE_M2L);
        fill_f64(Lx, 0.0, (int64_t)T.nbox * nb * PD, P->stream);
        {
            TranslateArgs a;
            a.cols_box = Y.m2l_cols;
            a.ncols = Y.n_m2l_cols * nb;
            a.nbatch = nb;
            a.slots = Y.m2l_slot;
            a.nops = NOFF * T.nlevels;
            a.tile_ptr = Y.m2l_tptr;
            a.tile_ops = Y.m2l_tops;
            a.tile_order = Y.m2l_torder;
            a.in = ex;
            a.out = ex;
            a.nrows_out = PD;
            a.logrow = -1;
            a.level = T.level;
            a.logside = T.d_logside;
            a.zero_col = P->zero_col;
            const unsigned grid = (unsigned)((a.ncols + 15) / 16);
            switch (PD) {
#define VP_YL(RB)                                                                                                 \
    case RB * 16:                                                                                                 \
        hipLaunchKernelGGL((k_translate_split<double, double, double, RB, RB * 4, false, true>), dim3(grid),       \
                           dim3(256), 0, P->stream, a, Y.m2l, (const double *)nullptr, M, Lx);                   \
        break;
                VP_YL(1) VP_YL(2) VP_YL(3) VP_YL(4)
#undef VP_YL
            }
            VP_LAUNCH_CHECK();
        }
        P->stage_end(VP_STAGE_M2L);
        // L2L, coarsest first (add into the children)
        P->stage_begin(VP_STAGE_L2L);
        for (int l = 2; l + 1 <= L; ++l)
            gemm(Y.d_children[l + 1], (int)Y.children[l + 1].size(), Y.pslot, Y.l2l + (size_t)l * 4 * AE, Lx, Lx,
                 true);
        P->stage_end(VP_STAGE_L2L);
        // pattern L2P of the leaves (store)
        P->stage_begin(VP_STAGE_FAR);
        {
            const ColAddr pout{R.ntgt, 0, R.tb};
            switch (PD) {
#define VP_YQ(RB)                                                                                                 \
    case RB * 16:                                                                                                 \
        launch_fixed_apply<double, double, double, 4, RB * 4, false>(P, N.l2p_pat, N.n_l2p_pat * nb, ex, pout, 64, \
                                                                     Y.l2p, Lx, P->acc_far);                      \
        break;
                VP_YQ(1) VP_YQ(2) VP_YQ(3) VP_YQ(4)
#undef VP_YQ
            }
        }
        P->stage_end(VP_STAGE_FAR);
    }
    if (u) add_fmm_sums(P, u, adjoint);
}

void run_fmm(vp_plan_s *P, bool adjoint, bool grad, const double *f, double *u) {
    PointRoles R = roles(P, adjoint);
    BoxGeo G = geo(P);
    if (P->yk.active) {
        run_yukawa(P, R, adjoint, f, u);
        return;
    }
    if (P->fp32) run_passes<float>(P, R, G, adjoint, grad, f, u);
    else run_passes<double>(P, R, G, adjoint, grad, f, u);
}

// The sparse correction (Section 4): out = C f (adjoint: C^T g), on the
// current stream; it needs no FMM result, so it runs beside the expansions.
static void correction_apply(vp_plan_s *P, const double *f, double *u, bool adjoint) {
    const int64_t nrows = adjoint ? P->nd : P->m;
    const int64_t *rp = adjoint ? P->rowptrT : P->rowptr;
    const int32_t *cv = adjoint ? P->colT : P->col;
    const int32_t *rs = adjoint ? P->run_startT : P->run_start;
    const double *vv = adjoint ? P->valT : P->val;
    const bool runs = adjoint ? P->all_runsT : P->all_runs;
    const int64_t flen = adjoint ? P->m : P->nd;
    int64_t blocks = (nrows * 16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    const int ncell = adjoint ? P->ncellT : P->ncell;
    const double *cop = adjoint ? P->corr_opT : P->corr_op;
    P->stage_begin(VP_STAGE_CORR);
    if (P->nnz == 0) {
        fill_f64(u, 0.0, (int64_t)P->nbatch * nrows, P->stream);
    } else if (ncell > 0 && cop) {
        // one shared 64 x 64 block: u[b][row0 + r] = sum_j V[r][j] f[b][col0 + j] per cell
        const int32_t *crow = adjoint ? P->cell_rowT : P->cell_row;
        const int32_t *ccol = adjoint ? P->cell_colT : P->cell_col;
        launch_fixed_apply<double, double, double, 4, 16, false>(P, P->cell_iota, ncell * P->nbatch,
                                                                 ColAddr{flen, 0, ccol}, ColAddr{nrows, 0, crow}, 64,
                                                                 cop, f, u);
    } else if (ncell > 0) {
        const int32_t *crow = adjoint ? P->cell_rowT : P->cell_row;
        const int32_t *ccol = adjoint ? P->cell_colT : P->cell_col;
        const int64_t *cvb = adjoint ? P->cell_vbT : P->cell_vb;
        const int ngrp = adjoint ? P->ngrpT : P->ngrp;
        if (P->nbatch == 1 && ngrp > 0) {
            // shared-block cells as groups on the matrix cores; the rest below
            cvb = adjoint ? P->cell_vbgT : P->cell_vbg;
            const unsigned gblocks = (unsigned)std::min<int64_t>((ngrp + 3) / 4, 16384);
            hipLaunchKernelGGL(k_corr_group, dim3(gblocks), dim3(256), 0, P->stream, ngrp,
                               adjoint ? P->grp_cellT : P->grp_cell, adjoint ? P->grp_vbT : P->grp_vb,
                               adjoint ? P->grp_rowsT : P->grp_rows, crow, ccol, vv, f, u);
            VP_LAUNCH_CHECK();
        }
        const unsigned cblocks = (unsigned)std::min<int64_t>((ncell + 3) / 4, 16384);
        for (int bt0 = 0; bt0 < P->nbatch;) {
            const int left = P->nbatch - bt0;
            const int g = left >= 16 ? 16 : (left >= 8 ? 8 : (left >= 4 ? 4 : (left >= 2 ? 2 : 1)));
            switch (g) {
#define VP_CELLS(G)                                                                                              \
    case G:                                                                                                      \
        hipLaunchKernelGGL((k_corr_cells<G>), dim3(cblocks), dim3(256), 0, P->stream, ncell, crow, ccol, cvb,    \
                           P->nbatch, bt0, rp, vv, f, flen, nrows, u);                                           \
        break;
                VP_CELLS(16) VP_CELLS(8) VP_CELLS(4) VP_CELLS(2) VP_CELLS(1)
#undef VP_CELLS
            }
            VP_LAUNCH_CHECK();
            bt0 += g;
        }
    } else {
        for (int bt0 = 0; bt0 < P->nbatch;) {
            const int left = P->nbatch - bt0;
            const int g = left >= 16 ? 16 : (left >= 8 ? 8 : (left >= 4 ? 4 : (left >= 2 ? 2 : 1)));
            switch (g) {
#define VP_FIN(G)                                                                                              \
    case G:                                                                                                    \
        if (runs)                                                                                              \
            hipLaunchKernelGGL((k_corr<G, true>), dim3((unsigned)blocks), dim3(256), 0, P->stream, nrows,      \
                               P->nbatch, bt0, (int64_t)P->nnz, rp, cv, rs, vv, f, flen, u);                   \
        else                                                                                                   \
            hipLaunchKernelGGL((k_corr<G, false>), dim3((unsigned)blocks), dim3(256), 0, P->stream, nrows,     \
                               P->nbatch, bt0, (int64_t)P->nnz, rp, cv, rs, vv, f, flen, u);                  \
        break;
                VP_FIN(16) VP_FIN(8) VP_FIN(4) VP_FIN(2) VP_FIN(1)
#undef VP_FIN
            }
            VP_LAUNCH_CHECK();
            bt0 += g;
        }
    }
    P->stage_end(VP_STAGE_CORR);
}

// out += (adjoint: w times) the FMM sums, un-permuted to user order
// (adjoint of an oversampled plan: O^T of the weighted sums per box)
static void add_fmm_sums(vp_plan_s *P, double *u, bool adjoint) {
    if (adjoint && P->os_p > 0) {
        P->stage_begin(VP_STAGE_FINISH);
        hipLaunchKernelGGL(k_interp_adjoint, dim3((unsigned)P->os_nbox), dim3(256), 0, P->stream, P->os_in,
                           P->os_out, P->os_p * P->os_p, P->os_q * P->os_q, P->os_O, P->acc, P->acc_far, P->n,
                           P->sinv, P->w_user, P->nbatch, P->nd, u);
        VP_LAUNCH_CHECK();
        P->stage_end(VP_STAGE_FINISH);
        return;
    }
    const int64_t nrows = adjoint ? P->n : P->m;
    const int32_t *inv = adjoint ? P->sinv : P->tinv;
    const double *scale = adjoint ? P->w_user : nullptr;
    P->stage_begin(VP_STAGE_FINISH);
    hipLaunchKernelGGL(k_add_acc, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0, P->stream, nrows, P->nbatch,
                       inv, scale, P->acc, P->acc_far, nrows, u);
    VP_LAUNCH_CHECK();
    P->stage_end(VP_STAGE_FINISH);
}

// Wall time of one full forward evaluation (the smallest of reps after one
// warm-up), on the plan's stream, with device buffers f and u.
float time_forward(vp_plan_s *P, const double *f, double *u, int reps) {
    hipEvent_t e0, e1;
    VP_HIP(hipEventCreate(&e0));
    VP_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    for (int rep = 0; rep <= reps; ++rep) {
        VP_HIP(hipEventRecord(e0, P->stream));
        prepare_charges(P, f, false);
        run_fmm(P, false, false, f, u);
        VP_HIP(hipEventRecord(e1, P->stream));
        VP_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        VP_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) best = std::min(best, ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

// Plan-time autotuner: coordinate descent over the evaluation's knobs, each
// candidate timed on full evaluations of this plan (density 1 everywhere):
//   M2L form       FP64: scaled, per-offset products;  FP32-bulk: scaled FP32,
//                  per-offset FP32, split hi/lo FP32, scaled FP64 (every one
//                  meets the precision's accuracy target)
//   M2L waves per 16-column tile (4, 2, or one wave per tile in the scaled
//   forms), near-table waves per tile (4, 2, or one wave over two tiles),
//   streams (three, one).
// Returns the best time (ms).
float autotune(vp_plan_s *P) {
    TempArena tmp;
    double *f = tmp.alloc<double>((size_t)P->nbatch * P->nd);
    double *u = tmp.alloc<double>((size_t)P->nbatch * P->m);
    fill_f64(f, 1.0, (int64_t)P->nbatch * P->nd, P->stream);
    int reps = 3;
    float best = time_forward(P, f, u, reps);
    // short evaluations (a fraction of a millisecond) vary by several percent
    // from one to the next: take the best of more of them, about 20 ms a candidate
    reps = std::max(3, std::min(15, (int)(20.f / std::max(best, 1e-3f))));
    if (reps > 3) best = std::min(best, time_forward(P, f, u, reps));
    auto knob = [&](int &field, const std::vector<int> &cand) {
        int keep = field;
        for (int v : cand) {
            if (v == keep) continue;
            field = v;
            const float t = time_forward(P, f, u, reps);
            if (t < best) {
                best = t;
                keep = v;
            }
        }
        field = keep;
    };
    if (P->fp32) knob(P->m2l_mode, {VP_M2L_FP32_SCALED, VP_M2L_FP32_MFMA, VP_M2L_FP32_SPLIT, VP_M2L_FP64_SCALED});
    else knob(P->m2l_mode, {VP_M2L_FP64_SCALED, VP_M2L_FP64_MFMA});
    if (P->opt.m2l_waves == 0) {
        const bool scaled = P->m2l_mode == VP_M2L_FP64_SCALED || P->m2l_mode == VP_M2L_FP32_SCALED;
        knob(P->m2l_nw, scaled ? std::vector<int>{1, 4, 2} : std::vector<int>{1, 2});
    }
    if (P->opt.table_waves == 0 && P->near.active) knob(P->table_nw, {1, 4, 2});
    int one = P->one_stream ? 1 : 0;
    if (!(P->opt.flags & VP_FLAG_ONE_STREAM)) {
        bool &fld = P->one_stream;
        for (int v : {0, 1}) {
            if (v == one) continue;
            fld = v != 0;
            const float t = time_forward(P, f, u, reps);
            if (t < best) {
                best = t;
                one = v;
            }
        }
        fld = one != 0;
    }
    VP_HIP(hipStreamSynchronize(P->stream));
    return best;
}

void finish_grad(vp_plan_s *P, double *grad) {
    P->stage_begin(VP_STAGE_FINISH);
    hipLaunchKernelGGL(k_unpermute_grad, dim3((unsigned)((P->m + 255) / 256)), dim3(256), 0, P->stream, P->m,
                       P->nbatch, P->tinv, P->acc, grad);
    VP_LAUNCH_CHECK();
    P->stage_end(VP_STAGE_FINISH);
}

}  // namespace vp

// Translation operators of the 2D Laplace FMM, precomputed once per plan in
// float64 on the host.
//
// Expansions are stored scaled by the box side s (level dependent) so that
// every operator is level independent:
//   multipole  phi(z) = A_0 log(z - c) + sum_k A_k (s/(z - c))^k,
//              A_0 = sum q, A_k = -(1/k) sum q ((z_j - c)/s)^k
//   local      phi(z) = sum_l B_l ((z - c)/s)^l
// and u = -(1/(2 pi)) Re phi (G of Section 2.1 in complex form).  The
// operators follow from the series of log(1 - x) and the binomial theorem:
//   M2M, child of side s1 at (c1 - c2) = s1 t into a parent of side 2 s1:
//       B_0 = A_0,  B_l = 2^-l [ -A_0 t^l / l + sum_{k=1..l} C(l-1,k-1) t^(l-k) A_k ]
//   M2L, boxes of side s, source centre - target centre = s t:
//       B_0 = A_0 (log s + log(-t)) + sum_k (-1)^k A_k / t^k
//       B_l = -A_0/(l t^l) + sum_k (-1)^k C(l+k-1,k-1) A_k / t^(l+k)
//   L2L, parent of side s2, child centre - parent centre = s2 t:
//       B'_l = 2^-l sum_{k>=l} C(k,l) t^(k-l) B_k
// A complex P x P operator T acts on the real column [Re a; Im a] (rows
// 0..P-1 real parts, P..2P-1 imaginary parts, zero padding to PD) as
// [[Re T, -Im T], [Im T, Re T]].  The M2L operators carry one more row,
// 2P, that sums Re A_0 so that the kernel can add A_0 log s for the
// level of each target box.

#include <cmath>
#include <complex>
#include <vector>

#include "vp_internal.hpp"

namespace vp {

using cd = std::complex<double>;

static std::vector<double> binom_table(int N) {
    std::vector<double> C((size_t)(N + 1) * (N + 1), 0.0);
    for (int a = 0; a <= N; ++a) {
        C[(size_t)a * (N + 1)] = 1.0;
        for (int b = 1; b <= a; ++b)
            C[(size_t)a * (N + 1) + b] = C[(size_t)(a - 1) * (N + 1) + b - 1] +
                                         (b <= a - 1 ? C[(size_t)(a - 1) * (N + 1) + b] : 0.0);
    }
    return C;
}

// complex P x P (row l, column k) -> real PD x PD row-major
static void to_real(const std::vector<cd> &T, int P, int PD, double *R) {
    for (int i = 0; i < PD * PD; ++i) R[i] = 0.0;
    for (int l = 0; l < P; ++l)
        for (int k = 0; k < P; ++k) {
            cd t = T[(size_t)l * P + k];
            R[(size_t)l * PD + k] = t.real();
            R[(size_t)l * PD + P + k] = -t.imag();
            R[(size_t)(P + l) * PD + k] = t.imag();
            R[(size_t)(P + l) * PD + P + k] = t.real();
        }
}

static std::vector<cd> m2l_complex(cd t, int P, const std::vector<double> &C, int N) {
    std::vector<cd> T((size_t)P * P, cd(0, 0));
    std::vector<cd> it(2 * P + 1);  // t^-n
    it[0] = 1.0;
    for (int n = 1; n <= 2 * P; ++n) it[n] = it[n - 1] / t;
    T[0] = std::log(-t);
    for (int k = 1; k < P; ++k) T[k] = ((k & 1) ? -1.0 : 1.0) * it[k];
    for (int l = 1; l < P; ++l) {
        T[(size_t)l * P] = -it[l] / (double)l;
        for (int k = 1; k < P; ++k)
            T[(size_t)l * P + k] = ((k & 1) ? -1.0 : 1.0) * C[(size_t)(l + k - 1) * (N + 1) + k - 1] * it[l + k];
    }
    return T;
}

// outer offsets in code order
static void offset_of_code(int code, int &dx, int &dy) {
    for (int y = -3; y <= 3; ++y)
        for (int x = -3; x <= 3; ++x)
            if (offset_code(x, y) == code) {
                dx = x;
                dy = y;
                return;
            }
    dx = dy = 0;
}

}  // namespace vp

// row-major rows x cols (leading dimension ld) -> MFMA A-fragment order
// [rb][s][lane]: element (row rb*16 + lane%16, col 4 s + lane/16)
void vp_to_frag(const double *R, int rows, int cols, int ld, double *F) {
    int RB = rows / 16, S = cols / 4;
    for (int rb = 0; rb < RB; ++rb)
        for (int s = 0; s < S; ++s)
            for (int lane = 0; lane < 64; ++lane)
                F[((size_t)rb * S + s) * 64 + lane] = R[(size_t)(rb * 16 + lane % 16) * ld + 4 * s + lane / 16];
}

// The same fragments with the k index split the other way: lane group g takes
// the S consecutive columns S g .. S g + S - 1 over the S steps (a lane's
// input elements are then contiguous: k_l2p_fin loads them 16 bytes at a time)
void vp_to_frag_kmajor(const double *R, int rows, int cols, int ld, double *F) {
    int RB = rows / 16, S = cols / 4;
    for (int rb = 0; rb < RB; ++rb)
        for (int s = 0; s < S; ++s)
            for (int lane = 0; lane < 64; ++lane)
                F[((size_t)rb * S + s) * 64 + lane] = R[(size_t)(rb * 16 + lane % 16) * ld + S * (lane / 16) + s];
}

namespace vp {

static void to_frag(const double *R, int PD, double *F) { vp_to_frag(R, PD, PD, PD, F); }

void build_operators(vp_plan_s *P) {
    const int Pn = P->P, PD = P->PD;
    const int N = 2 * Pn + 2;
    auto C = binom_table(N);
    Operators &O = P->ops;
    O.P = Pn;
    O.PD = PD;
    const size_t mat = (size_t)PD * PD;

    std::vector<double> R(mat), F((size_t)NOFF * mat);
    for (int code = 0; code < NOFF; ++code) {
        int dx, dy;
        offset_of_code(code, dx, dy);
        auto T = m2l_complex(cd(dx, dy), Pn, C, N);
        to_real(T, Pn, PD, R.data());
        R[(size_t)(2 * Pn) * PD + 0] = 1.0;  // sum of Re A_0 (log s term)
        to_frag(R.data(), PD, F.data() + code * mat);
    }
    // M2M and L2L in diagonally scaled form, per child class q (bit 0: +x, bit 1: +y):
    //   M2M, t = child offset / child side = (+-1/2, +-1/2):
    //       B_l = 2^-l t^l [ -A_0 / l + sum_{k=1..l} C(l-1, k-1) t^-k A_k ],  B_0 = A_0
    //   L2L, t = child offset / parent side = (+-1/4, +-1/4):
    //       B'_l = 2^-l t^-l sum_{k>=l} C(k, l) t^k B_k
    int PR = 16;
    while (PR < Pn) PR *= 2;
    O.PR = PR;
    std::vector<double> shq[2], shin[2], shout[2];
    for (int w = 0; w < 2; ++w) {
        shq[w].assign((size_t)Pn * PR, 0.0);
        shin[w].assign((size_t)4 * Pn * 2, 0.0);
        shout[w].assign((size_t)4 * Pn * 2, 0.0);
    }
    // QT[k][l] = Q[l][k]
    shq[0][0] = 1.0;
    for (int l = 1; l < Pn; ++l) {
        shq[0][(size_t)0 * PR + l] = -1.0 / l;
        for (int k = 1; k <= l; ++k) shq[0][(size_t)k * PR + l] = C[(size_t)(l - 1) * (N + 1) + k - 1];
    }
    for (int l = 0; l < Pn; ++l)
        for (int k = l; k < Pn; ++k) shq[1][(size_t)k * PR + l] = C[(size_t)k * (N + 1) + l];
    for (int q = 0; q < 4; ++q) {
        const double sx = (q & 1) ? 1.0 : -1.0, sy = (q >> 1) ? 1.0 : -1.0;
        const cd tm(0.5 * sx, 0.5 * sy), tl(0.25 * sx, 0.25 * sy);
        cd a_in = 1.0, a_out = 1.0, b_in = 1.0, b_out = 1.0;
        for (int k = 0; k < Pn; ++k) {
            const size_t e = ((size_t)q * Pn + k) * 2;
            shin[0][e] = a_in.real();
            shin[0][e + 1] = a_in.imag();
            shout[0][e] = a_out.real();
            shout[0][e + 1] = a_out.imag();
            shin[1][e] = b_in.real();
            shin[1][e + 1] = b_in.imag();
            shout[1][e] = b_out.real();
            shout[1][e + 1] = b_out.imag();
            a_in /= tm;          // t^-k
            a_out *= 0.5 * tm;   // 2^-l t^l
            b_in *= tl;          // t^k
            b_out /= 2.0 * tl;   // 2^-l t^-l
        }
    }
    // diagonally scaled M2L: Q with row l multiplied by (-1)^l, (-t)^-k and
    // log(-t) per offset (t^-l = (-1)^l (-t)^-l: one table scales both sides)
    const int PQ = (Pn + 15) / 16 * 16;
    O.PQ = PQ;
    std::vector<double> Qm((size_t)PQ * PQ, 0.0), Qf((size_t)PQ * PQ), tin((size_t)NOFF * PQ * 2, 0.0),
        logt(NOFF * 2);
    for (int k = 1; k < Pn; ++k) Qm[k] = 1.0;
    for (int l = 1; l < Pn; ++l) {
        const double sg = (l & 1) ? -1.0 : 1.0;
        Qm[(size_t)l * PQ] = sg * (-1.0 / l);
        for (int k = 1; k < Pn; ++k) Qm[(size_t)l * PQ + k] = sg * C[(size_t)(l + k - 1) * (N + 1) + k - 1];
    }
    vp_to_frag(Qm.data(), PQ, PQ, PQ, Qf.data());
    for (int code = 0; code < NOFF; ++code) {
        int dx, dy;
        offset_of_code(code, dx, dy);
        const cd t(dx, dy);
        cd pin = 1.0;
        for (int k = 0; k < Pn; ++k) {
            tin[((size_t)code * PQ + k) * 2] = pin.real();
            tin[((size_t)code * PQ + k) * 2 + 1] = pin.imag();
            pin /= -t;
        }
        const cd lg = std::log(-t);
        logt[2 * code] = lg.real();
        logt[2 * code + 1] = lg.imag();
    }
    // logarithm table of the pairwise near field: m in [1/2, 1) with top fraction
    // bits i lies in [1/2 + i/(2 LOG_TABLE), 1/2 + (i+1)/(2 LOG_TABLE)); c_i is
    // that interval's centre
    std::vector<double> ltab(2 * LOG_TABLE);
    for (int i = 0; i < LOG_TABLE; ++i) {
        const double c = 0.5 + (i + 0.5) / (2.0 * LOG_TABLE);
        const double inv_c = 1.0 / c;
        ltab[2 * i] = inv_c;
        ltab[2 * i + 1] = (double)(-log2l((long double)inv_c));
    }
    std::vector<double> invk(Pn, 0.0);
    for (int k = 1; k < Pn; ++k) invk[k] = 1.0 / k;

    hipStream_t s = P->stream;
    auto up = [&](const std::vector<double> &h) {
        double *d = P->mem.alloc<double>(h.size());
        VP_HIP(hipMemcpyAsync(d, h.data(), 8 * h.size(), hipMemcpyHostToDevice, s));
        return d;
    };
    auto upf = [&](const std::vector<float> &h) {
        float *d = P->mem.alloc<float>(h.size());
        VP_HIP(hipMemcpyAsync(d, h.data(), 4 * h.size(), hipMemcpyHostToDevice, s));
        return d;
    };
    O.m2l_f64 = up(F);
    for (int w = 0; w < 2; ++w) {
        O.sh_qt64[w] = up(shq[w]);
        O.sh_tin64[w] = up(shin[w]);
        O.sh_tout64[w] = up(shout[w]);
    }
    O.inv_k = up(invk);
    O.log_table = up(ltab);
    O.m2l_q64 = up(Qf);
    O.m2l_tin64 = up(tin);
    O.m2l_logt = up(logt);
    // host copies must outlive the asynchronous uploads (synchronised below)
    std::vector<float> q32(Qf.begin(), Qf.end()), tin32(tin.begin(), tin.end());
    if (P->fp32) {
        O.m2l_q32 = upf(q32);
        O.m2l_tin32 = upf(tin32);
        std::vector<float> hi(F.size()), lo(F.size());
        for (size_t i = 0; i < F.size(); ++i) {
            hi[i] = (float)F[i];
            lo[i] = (float)(F[i] - (double)hi[i]);
        }
        O.m2l_f32 = upf(hi);
        O.m2l_f32_lo = upf(lo);
        std::vector<float> c(invk.begin(), invk.end());
        O.inv_k_f32 = upf(c);
        std::vector<float> fq[2], fi[2], fo[2];
        for (int w = 0; w < 2; ++w) {
            fq[w].assign(shq[w].begin(), shq[w].end());
            fi[w].assign(shin[w].begin(), shin[w].end());
            fo[w].assign(shout[w].begin(), shout[w].end());
            O.sh_qt32[w] = upf(fq[w]);
            O.sh_tin32[w] = upf(fi[w]);
            O.sh_tout32[w] = upf(fo[w]);
        }
        VP_HIP(hipStreamSynchronize(s));  // before the host copies above go out of scope
    }
    VP_HIP(hipStreamSynchronize(s));
}

}  // namespace vp

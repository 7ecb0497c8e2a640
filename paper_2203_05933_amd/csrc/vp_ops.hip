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

static std::vector<cd> m2m_complex(cd t, int P, const std::vector<double> &C, int N) {
    std::vector<cd> T((size_t)P * P, cd(0, 0));
    std::vector<cd> tp(P + 1);
    tp[0] = 1.0;
    for (int n = 1; n <= P; ++n) tp[n] = tp[n - 1] * t;
    T[0] = 1.0;
    for (int l = 1; l < P; ++l) {
        double sc = std::ldexp(1.0, -l);
        T[(size_t)l * P] = -tp[l] / (double)l * sc;
        for (int k = 1; k <= l; ++k)
            T[(size_t)l * P + k] = C[(size_t)(l - 1) * (N + 1) + k - 1] * tp[l - k] * sc;
    }
    return T;
}

static std::vector<cd> l2l_complex(cd t, int P, const std::vector<double> &C, int N) {
    std::vector<cd> T((size_t)P * P, cd(0, 0));
    std::vector<cd> tp(P + 1);
    tp[0] = 1.0;
    for (int n = 1; n <= P; ++n) tp[n] = tp[n - 1] * t;
    for (int l = 0; l < P; ++l) {
        double sc = std::ldexp(1.0, -l);
        for (int k = l; k < P; ++k) T[(size_t)l * P + k] = C[(size_t)k * (N + 1) + l] * tp[k - l] * sc;
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
    std::vector<double> M2M(4 * mat), L2L(4 * mat), M2Mt(4 * mat), L2Lt(4 * mat);
    auto transpose = [&](const double *Rm, double *out) {
        for (int r = 0; r < PD; ++r)
            for (int k = 0; k < PD; ++k) out[(size_t)k * PD + r] = Rm[(size_t)r * PD + k];
    };
    for (int q = 0; q < 4; ++q) {
        double sx = (q & 1) ? 1.0 : -1.0, sy = (q >> 1) ? 1.0 : -1.0;
        auto Tm = m2m_complex(cd(0.5 * sx, 0.5 * sy), Pn, C, N);
        to_real(Tm, Pn, PD, R.data());
        to_frag(R.data(), PD, M2M.data() + q * mat);
        transpose(R.data(), M2Mt.data() + q * mat);
        auto Tl = l2l_complex(cd(0.25 * sx, 0.25 * sy), Pn, C, N);
        to_real(Tl, Pn, PD, R.data());
        to_frag(R.data(), PD, L2L.data() + q * mat);
        transpose(R.data(), L2Lt.data() + q * mat);
    }
    // diagonally scaled M2L: Q, (-t)^-k, t^-l and log(-t) per offset
    const int PQ = (Pn + 15) / 16 * 16;
    O.PQ = PQ;
    std::vector<double> Qm((size_t)PQ * PQ, 0.0), Qf((size_t)PQ * PQ), tin((size_t)NOFF * PQ * 2, 0.0),
        tout((size_t)NOFF * PQ * 2, 0.0), logt(NOFF * 2);
    for (int k = 1; k < Pn; ++k) Qm[k] = 1.0;
    for (int l = 1; l < Pn; ++l) {
        Qm[(size_t)l * PQ] = -1.0 / l;
        for (int k = 1; k < Pn; ++k) Qm[(size_t)l * PQ + k] = C[(size_t)(l + k - 1) * (N + 1) + k - 1];
    }
    vp_to_frag(Qm.data(), PQ, PQ, PQ, Qf.data());
    for (int code = 0; code < NOFF; ++code) {
        int dx, dy;
        offset_of_code(code, dx, dy);
        const cd t(dx, dy);
        cd pin = 1.0, pout = 1.0;
        for (int k = 0; k < Pn; ++k) {
            tin[((size_t)code * PQ + k) * 2] = pin.real();
            tin[((size_t)code * PQ + k) * 2 + 1] = pin.imag();
            tout[((size_t)code * PQ + k) * 2] = pout.real();
            tout[((size_t)code * PQ + k) * 2 + 1] = pout.imag();
            pin /= -t;
            pout /= t;
        }
        const cd lg = std::log(-t);
        logt[2 * code] = lg.real();
        logt[2 * code + 1] = lg.imag();
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
    O.m2m_f64 = up(M2M);
    O.l2l_f64 = up(L2L);
    O.m2m_t64 = up(M2Mt);
    O.l2l_t64 = up(L2Lt);
    O.inv_k = up(invk);
    O.m2l_q64 = up(Qf);
    O.m2l_tin64 = up(tin);
    O.m2l_tout64 = up(tout);
    O.m2l_logt = up(logt);
    // host copies must outlive the asynchronous uploads (synchronised below)
    std::vector<float> q32(Qf.begin(), Qf.end()), tin32(tin.begin(), tin.end()), tout32(tout.begin(), tout.end());
    if (P->fp32) {
        O.m2l_q32 = upf(q32);
        O.m2l_tin32 = upf(tin32);
        O.m2l_tout32 = upf(tout32);
        std::vector<float> hi(F.size()), lo(F.size());
        for (size_t i = 0; i < F.size(); ++i) {
            hi[i] = (float)F[i];
            lo[i] = (float)(F[i] - (double)hi[i]);
        }
        O.m2l_f32 = upf(hi);
        O.m2l_f32_lo = upf(lo);
        std::vector<float> a(M2M.begin(), M2M.end()), b(L2L.begin(), L2L.end()), c(invk.begin(), invk.end());
        O.m2m_f32 = upf(a);
        O.l2l_f32 = upf(b);
        std::vector<float> at(M2Mt.begin(), M2Mt.end()), bt(L2Lt.begin(), L2Lt.end());
        O.m2m_t32 = upf(at);
        O.l2l_t32 = upf(bt);
        O.inv_k_f32 = upf(c);
        VP_HIP(hipStreamSynchronize(s));  // before the host copies above go out of scope
    }
    VP_HIP(hipStreamSynchronize(s));
}

}  // namespace vp

// Modified Helmholtz (Yukawa) kernel: plan-time operators.
//
// Section 2.1 gives the Green's function of L = -Delta + lambda^2 as
// G(r, r0) = (lambda^2 / 2 pi) K_0(lambda |r - r0|); the smooth rule of
// Section 3.2 (eq. Tk_smooth_quad) is the same point sum with it, and
// Section 5 runs the modified Helmholtz experiment (lambda^2 = 100).  The
// FMM for this kernel uses the expansions of the addition theorem for
// modified Bessel functions, in complex notation K_n(d) = K_|n|(lambda |d|)
// e^{i n arg d}, I_n(d) likewise (z the complex position, c a box centre):
//   multipole  phi(z) = sum_{|n|<=p} a_n K_n(z - c),   a_n = sum_j q_j conj(I_n(z_j - c))
//   local      psi(z) = sum_{|n|<=p} b_n I_n(z - c),   b_n = sum_j q_j conj(K_n(z_j - c))
//   M2M  (child c1 -> parent c2)      a'_k = sum_n a_n I_{n-k}(c1 - c2)
//   M2L  (source c1 -> target c3)     b_m  = (-1)^m sum_n a_n K_{n-m}(c3 - c1)
//   L2L  (parent c2 -> child c3)      b'_m = sum_n b_n I_{n-m}(c3 - c2)
//   L2P                               u(z) = lambda^2/(2 pi) sum_n b_n I_n(z - c)
// A real field has a_{-n} = conj(a_n) (K_{-n}(d) = conj K_n(d) for real order
// functions), so a column stores n = 0..p as [Re a; Im a] like the Laplace
// expansions, and each operator is a real 2P x 2P matrix (built by applying
// the formula to the real basis vectors; the map involves conjugates, so it
// is real-linear rather than complex-linear).  To keep the coefficients of
// every level near unit size, the stored coefficients are scaled by the
// level's box side h: a^_n = a_n / I_n(lambda h), b^_n = b_n I_n(lambda h).
//
// Everything here is a fixed matrix: on a uniform grid of congruent leaves
// (one leaf level, no W or X lists, every near pair served by a table) the
// whole evaluation is the near tables (G at the pattern offsets), the
// pattern P2M and L2P, and per level the M2M, M2L and L2L operators, all
// applied by the matrix-core kernels that serve the Laplace kernel.  The
// Bessel functions are evaluated in long double on the host (vp_bessel.hpp).

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "vp_bessel.hpp"
#include "vp_internal.hpp"

namespace vp {

using cld = std::complex<long double>;

namespace {

template <class T>
T *upload_vec(vp_plan_s *P, const std::vector<T> &h) {
    T *d = P->mem.alloc<T>(h.size());
    if (!h.empty()) VP_HIP(hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, P->stream));
    return d;
}

// Bessel values at one argument times the phase: f_|k|(lambda |d|) e^{i k arg d},
// k = -kmax..kmax, tabulated once per argument
struct BesselRow {
    std::vector<cld> v;  // index k + kmax
    int kmax = 0;
    cld at(int k) const { return v[(size_t)(k + kmax)]; }
};

BesselRow bessel_row(bool kind_k, long double lam, cld d, int kmax) {
    std::vector<long double> f((size_t)kmax + 1);
    const long double x = lam * std::abs(d);
    if (kind_k) bessel_k_all(x, kmax, f.data());
    else bessel_i_all(x, kmax, f.data());
    const long double arg = std::arg(d);
    BesselRow r;
    r.kmax = kmax;
    r.v.resize((size_t)2 * kmax + 1);
    for (int k = -kmax; k <= kmax; ++k) {
        const long double a = (long double)k * arg;
        r.v[(size_t)(k + kmax)] = f[(size_t)std::abs(k)] * cld(std::cos(a), std::sin(a));
    }
    return r;
}

// Real 2P x 2P form (PD x PD row-major, zero padded) of a real-linear map
// from coefficients a_n (n = 0..p, a_{-n} = conj a_n) to b_m (m = 0..p).
template <class F>
void real_form(int P, int PD, F &&apply, std::vector<double> &R) {
    R.assign((size_t)PD * PD, 0.0);
    std::vector<cld> a((size_t)2 * P - 1), b((size_t)P);
    for (int c = 0; c < 2 * P; ++c) {
        const int n = c < P ? c : c - P;
        if (c == P) continue;  // Im a_0 of a real field is zero
        std::fill(a.begin(), a.end(), cld(0, 0));
        const cld unit = c < P ? cld(1, 0) : cld(0, 1);
        a[(size_t)(n + P - 1)] = unit;                      // a_n
        if (n > 0) a[(size_t)(P - 1 - n)] = std::conj(unit);  // a_{-n}
        apply(a, b);  // a indexed n + p (p = P - 1)
        for (int m = 0; m < P; ++m) {
            R[(size_t)m * PD + c] = (double)b[(size_t)m].real();
            R[(size_t)(P + m) * PD + c] = (double)b[(size_t)m].imag();
        }
    }
}

}  // namespace

void build_yukawa(vp_plan_s *P) {
    YukawaPlan &Y = P->yk;
    Tree &T = P->tree;
    NearTables &N = P->near;
    hipStream_t s = P->stream;
    const int nbox = T.nbox, Pn = P->P, PD = P->PD, p = Pn - 1;
    const long double lam = P->opt.lambda;
    Y.lambda = (double)lam;
    Y.cG = (double)(lam * lam / (2.0L * 3.141592653589793238462643383279502884L));

    std::vector<int32_t> lev(nbox), ix(nbox), iy(nbox), nch(nbox), par(nbox), leaves(T.nleaf);
    VP_HIP(hipMemcpyAsync(lev.data(), T.level, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(ix.data(), T.ix, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(iy.data(), T.iy, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(nch.data(), T.nchild, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(par.data(), T.parent, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(leaves.data(), T.leaves, 4 * T.nleaf, hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));

    // --- what this build supports: a uniform grid of congruent leaves
    auto unsupported = [](const std::string &m) {
        throw Error(VP_EUNSUPPORTED, "modified Helmholtz kernel: " + m);
    };
    if (!N.active || N.npat != 64) unsupported("needs leaves that all carry one 64-point node pattern (targets = nodes)");
    int L = -1;
    for (int b : leaves) {
        if (L < 0) L = lev[b];
        if (lev[b] != L) unsupported("needs every leaf on one level (a uniform grid of boxes)");
    }
    if (L >= 2 && N.n_l2p_pat != (int)leaves.size()) unsupported("needs every leaf to match the node pattern");
    if (T.llen[2] != 0 || T.llen[3] != 0) unsupported("needs a tree without W and X lists");
    if (N.rest_len != 0 || N.n_zero_near != 0) unsupported("needs every near pair served by a table");
    if (PD > 64) unsupported("order too large (p + 1 <= 32)");
    Y.active = true;
    Y.leaf_level = L;
    const int nlev = T.nlevels;

    // --- near-field tables: the Laplace tables' slots, filled with this kernel
    {
        const int np = N.npat;
        const std::vector<double> &rx = N.pat_rx, &ry = N.pat_ry;
        std::vector<double> K((size_t)N.tab_levels.size() * NTOPS * np * np, 0.0), R((size_t)np * np);
        for (size_t li = 0; li < N.tab_levels.size(); ++li) {
            const long double h = T.side[N.tab_levels[li]];
            for (int o = 0; o < 9; ++o) {  // one leaf level: only same-level slots occur
                long double cxo, cyo, m;
                if (o < 9) {
                    cxo = (o % 3) - 1;
                    cyo = (o / 3) - 1;
                    m = 1.0L;
                } else if (o < 25) {
                    cxo = ((o - 9) % 4 - 2) + 0.5L;
                    cyo = ((o - 9) / 4 - 2) + 0.5L;
                    m = 2.0L;
                } else {
                    cxo = (((o - 25) % 4 - 1) - 0.5L) * 0.5L;
                    cyo = (((o - 25) / 4 - 1) - 0.5L) * 0.5L;
                    m = 0.5L;
                }
                for (int i = 0; i < np; ++i)
                    for (int j = 0; j < np; ++j) {
                        const long double ex = cxo + m * rx[j] - rx[i], ey = cyo + m * ry[j] - ry[i];
                        const long double r = h * std::sqrt(ex * ex + ey * ey);
                        long double k0 = 0, k1 = 0;
                        if (r > 0) bessel_k01(lam * r, k0, k1);
                        R[(size_t)i * np + j] = r > 0 ? (double)((long double)Y.cG * k0) : 0.0;
                    }
                vp_to_frag(R.data(), np, np, np, K.data() + ((size_t)li * NTOPS + o) * np * np);
            }
        }
        N.K = upload_vec(P, K);
        VP_HIP(hipStreamSynchronize(s));

        // pattern P2M (rows = expansion, cols = points) and L2P (rows = points,
        // cols = expansion) at the leaf level
        const long double hL = T.side[L];
        std::vector<long double> sc((size_t)Pn);
        bessel_i_all(lam * hL, p, sc.data());
        std::vector<double> A((size_t)PD * np, 0.0), B((size_t)np * PD, 0.0);
        for (int j = 0; j < np; ++j) {
            const cld d(hL * rx[j], hL * ry[j]);
            BesselRow I = bessel_row(false, lam, d, p);
            for (int n = 0; n <= p; ++n) {
                const cld v = std::conj(I.at(n)) / sc[(size_t)n];  // a^_n of a unit charge
                A[(size_t)n * np + j] = (double)v.real();
                A[(size_t)(Pn + n) * np + j] = (double)v.imag();
                // u = cG sum_{|n|<=p} b_n I_n(d), b_n = b^_n / sc_n, b_{-n} = conj b_n
                const long double mult = n == 0 ? 1.0L : 2.0L;
                const cld w = I.at(n) * (long double)Y.cG * mult / sc[(size_t)n];
                B[(size_t)j * PD + n] = (double)w.real();          // Re b^_n
                B[(size_t)j * PD + Pn + n] = (double)(-w.imag());  // Im b^_n
            }
        }
        std::vector<double> Af((size_t)PD * np), Bf((size_t)np * PD);
        vp_to_frag(A.data(), PD, np, np, Af.data());
        vp_to_frag(B.data(), np, PD, PD, Bf.data());
        Y.p2m = upload_vec(P, Af);
        Y.l2p = upload_vec(P, Bf);
        VP_HIP(hipStreamSynchronize(s));
    }

    // --- per-level scalings I_n(lambda h_l)
    std::vector<std::vector<long double>> sI(nlev, std::vector<long double>((size_t)Pn));
    for (int l = 0; l < nlev; ++l) bessel_i_all(lam * (long double)T.side[l], p, sI[l].data());

    const size_t AE = (size_t)PD * PD;
    std::vector<double> R, F(AE);
    auto at = [&](const std::vector<cld> &a, int n) { return a[(size_t)(n + p)]; };

    // --- M2M [parent level][child quadrant] and L2L [parent level][child quadrant]
    std::vector<double> m2m((size_t)nlev * 4 * AE, 0.0), l2l((size_t)nlev * 4 * AE, 0.0);
    for (int l = 2; l + 1 < nlev; ++l) {
        const long double hc = T.side[l + 1];
        for (int q = 0; q < 4; ++q) {
            const cld delta((q & 1) ? hc / 2 : -hc / 2, (q & 2) ? hc / 2 : -hc / 2);  // child - parent
            const BesselRow I = bessel_row(false, lam, delta, 2 * p);
            // M2M: a'_k = sum_n a_n I_{n-k}(delta), scaled child -> parent
            real_form(Pn, PD, [&](const std::vector<cld> &a, std::vector<cld> &b) {
                for (int k = 0; k <= p; ++k) {
                    cld acc(0, 0);
                    for (int n = -p; n <= p; ++n) acc += at(a, n) * sI[l + 1][(size_t)std::abs(n)] * I.at(n - k);
                    b[(size_t)k] = acc / sI[l][(size_t)k];
                }
            }, R);
            vp_to_frag(R.data(), PD, PD, PD, F.data());
            std::copy(F.begin(), F.end(), m2m.begin() + ((size_t)l * 4 + q) * AE);
            // L2L: b'_m = sum_n b_n I_{n-m}(delta), scaled parent -> child
            real_form(Pn, PD, [&](const std::vector<cld> &a, std::vector<cld> &b) {
                for (int m = 0; m <= p; ++m) {
                    cld acc(0, 0);
                    for (int n = -p; n <= p; ++n) acc += at(a, n) / sI[l][(size_t)std::abs(n)] * I.at(n - m);
                    b[(size_t)m] = acc * sI[l + 1][(size_t)m];
                }
            }, R);
            vp_to_frag(R.data(), PD, PD, PD, F.data());
            std::copy(F.begin(), F.end(), l2l.begin() + ((size_t)l * 4 + q) * AE);
        }
    }
    // --- M2L [level][offset code]: source = target + h (dx, dy)
    std::vector<double> m2l((size_t)nlev * NOFF * AE, 0.0);
    for (int l = 2; l < nlev; ++l) {
        const long double h = T.side[l];
        for (int dy = -3; dy <= 3; ++dy)
            for (int dx = -3; dx <= 3; ++dx) {
                const int code = offset_code(dx, dy);
                if (code < 0) continue;
                const cld d(-h * dx, -h * dy);  // target - source
                const BesselRow Kr = bessel_row(true, lam, d, 2 * p);
                real_form(Pn, PD, [&](const std::vector<cld> &a, std::vector<cld> &b) {
                    for (int m = 0; m <= p; ++m) {
                        cld acc(0, 0);
                        for (int n = -p; n <= p; ++n) acc += at(a, n) * sI[l][(size_t)std::abs(n)] * Kr.at(n - m);
                        b[(size_t)m] = ((m & 1) ? -1.0L : 1.0L) * acc * sI[l][(size_t)m];
                    }
                }, R);
                vp_to_frag(R.data(), PD, PD, PD, F.data());
                std::copy(F.begin(), F.end(), m2l.begin() + ((size_t)l * NOFF + code) * AE);
            }
    }
    Y.m2m = upload_vec(P, m2m);
    Y.l2l = upload_vec(P, l2l);
    Y.m2l = upload_vec(P, m2l);
    VP_HIP(hipStreamSynchronize(s));

    // --- slots and launch lists
    std::vector<int32_t> cslot((size_t)nbox * 4, -1), pslot((size_t)nbox * 4, -1);
    Y.parents.assign(nlev, {});
    Y.children.assign(nlev, {});
    for (int b = 0; b < nbox; ++b) {
        if (lev[b] >= 3) {
            const int q = (ix[b] & 1) | ((iy[b] & 1) << 1);
            cslot[(size_t)par[b] * 4 + q] = b;
            pslot[(size_t)b * 4 + q] = par[b];
            Y.children[lev[b]].push_back(b);
        }
    }
    for (int b = 0; b < nbox; ++b)
        if (lev[b] >= 2 && nch[b] > 0) Y.parents[lev[b]].push_back(b);
    Y.cslot = upload_vec(P, cslot);
    Y.pslot = upload_vec(P, pslot);
    Y.d_parents.assign(nlev, nullptr);
    Y.d_children.assign(nlev, nullptr);
    for (int l = 0; l < nlev; ++l) {
        if (!Y.parents[l].empty()) Y.d_parents[l] = upload_vec(P, Y.parents[l]);
        if (!Y.children[l].empty()) Y.d_children[l] = upload_vec(P, Y.children[l]);
    }
    // M2L: one slot row per box spanning all levels (the box's level block
    // holds its V-list sources), columns = boxes of level >= 2 by level
    std::vector<int32_t> vslot((size_t)nbox * NOFF);
    VP_HIP(hipMemcpyAsync(vslot.data(), T.v_slot, 4 * vslot.size(), hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));
    const size_t wrow = (size_t)NOFF * nlev;
    std::vector<int32_t> wide((size_t)nbox * wrow, -1), cols;
    for (int l = 2; l < nlev; ++l)
        for (int b = 0; b < nbox; ++b)
            if (lev[b] == l) {
                cols.push_back(b);
                for (int o = 0; o < NOFF; ++o) {
                    const int a = vslot[(size_t)b * NOFF + o];
                    if (a >= nbox) unsupported("needs a tree without X lists");
                    wide[(size_t)b * wrow + (size_t)l * NOFF + o] = a;
                }
            }
    const int64_t ncols = (int64_t)cols.size() * P->nbatch;
    std::vector<int32_t> tptr(1, 0), tops;
    std::vector<char> seen(wrow);
    int64_t trans = 0;
    for (int b : cols)
        for (int o = 0; o < NOFF; ++o) trans += vslot[(size_t)b * NOFF + o] >= 0;
    for (int64_t t = 0; t * 16 < ncols; ++t) {
        std::fill(seen.begin(), seen.end(), 0);
        for (int64_t c = 16 * t; c < std::min(ncols, 16 * t + 16); ++c) {
            const int b = cols[(size_t)(c / P->nbatch)];
            for (size_t o = 0; o < wrow; ++o)
                if (wide[(size_t)b * wrow + o] >= 0) seen[o] = 1;
        }
        for (size_t o = 0; o < wrow; ++o)
            if (seen[o]) tops.push_back((int32_t)o);
        tptr.push_back((int32_t)tops.size());
    }
    Y.n_m2l_cols = (int)cols.size();
    Y.m2l_cols = upload_vec(P, cols);
    Y.m2l_slot = upload_vec(P, wide);
    Y.m2l_tptr = upload_vec(P, tptr);
    Y.m2l_tops = upload_vec(P, tops);
    Y.m2l_torder = upload_vec(P, tile_order_by_work(tptr));
    Y.m2l_translations = trans;
    Y.m2l_tile_ops = (int64_t)tops.size();
    VP_HIP(hipStreamSynchronize(s));  // the host vectors leave scope
}

}  // namespace vp

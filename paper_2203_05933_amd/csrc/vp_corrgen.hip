// Own-cell singular corrections generated on the device (Section 4.1, eqs.
// maptri_singular_quad and singcorr_inner_prod; Section 4.2, eqs.
// mapbox_singular_quad and Vkhat_box).
//
// A cell is the affine image r = o + A zeta of a reference cell (the box
// [-1,1]^2, or the simplex xi, eta >= 0, xi + eta <= 1) carrying one node
// pattern zeta_j; the block of cell k is
//     C_ij = int_cell G(r, r_i) l_j(r) dA - [j != i] G(r_j, r_i) |det A| wref_j,
// l_j the Lagrange basis of the pattern's interpolation space.  With an
// orthogonal basis phi_n of that space (Legendre products on the box; on
// the simplex the collapsed-coordinate basis of Koornwinder's construction,
// P_a(c / t) t^a P_b^(2a+1,0)(2 eta - 1), c = 2 xi + eta - 1, t = 1 - eta) and
// V_jn = phi_n(zeta_j), l_j = sum_n phi_n (V^-1)_nj, so row i of the block is
// Vhat_i V^-1 less the smooth terms, Vhat_in = int G(r, r_i) phi_n dA.
//
// Singular rule.  The reference cell is split at zeta_i into triangles with
// apex zeta_i, one per edge P -> Q.  On each, zeta = zeta_i + u d(v),
// d(v) = (P - zeta_i) + v (Q - P), u, v in [0, 1], dzeta = u |d0 x d1| du dv,
// and since A (zeta - zeta_i) = u A d(v),
//     log|A (zeta - zeta_i)| = log u + log|A d(v)|
// exactly: the u integral of u (log u + c) times a polynomial in u is exact
// with 16 Gauss-Legendre points carrying two weight sets (u, and u log u by
// interpolation at those points; polynomials of degree < 16 along the ray),
// and the v integral is composite 12-point Gauss-Legendre, graded by factors
// of two toward the point of the edge nearest the target in PHYSICAL space
// (|A d(v)| is smallest there: a complex singularity of log|A d(v)| at
// v* +- i delta), with a first panel of half-width delta / 2.  The rule's
// points depend on the target's reference position and, through the grading,
// on the cell's shape; the cell enters through log|A d(v)| and |det A|.
#include <cmath>
#include <vector>

#include "vp_internal.hpp"

namespace vp {

namespace {

constexpr int NU = 16;  // Gauss-Legendre points along u
constexpr int NV = 12;  // Gauss-Legendre points per v panel

// n-point Gauss-Legendre on [-1, 1] in long double (Newton on P_n)
void gauss_legendre(int n, std::vector<long double> &x, std::vector<long double> &w) {
    x.assign(n, 0.0L);
    w.assign(n, 0.0L);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        long double z = std::cos(pi * (i + 0.75L) / (n + 0.5L)), dp = 0.0L;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1.0L, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) p1 = z, p0 = 1.0L;
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            const long double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-21L) break;
        }
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0L / ((1.0L - z * z) * dp * dp);
    }
}

// basis values phi_n(xi, eta) on the host, the same polynomials as on the device
void basis_host(int shape, int p, long double xi, long double eta, long double *out) {
    if (shape == 0) {
        std::vector<long double> Lx(p), Ly(p);
        for (int k = 0; k < p; ++k) {
            if (k == 0) Lx[k] = Ly[k] = 1.0L;
            else if (k == 1) Lx[k] = xi, Ly[k] = eta;
            else {
                Lx[k] = ((2 * k - 1) * xi * Lx[k - 1] - (k - 1) * Lx[k - 2]) / k;
                Ly[k] = ((2 * k - 1) * eta * Ly[k - 1] - (k - 1) * Ly[k - 2]) / k;
            }
        }
        for (int a = 0; a < p; ++a)
            for (int b = 0; b < p; ++b) out[a * p + b] = Lx[a] * Ly[b];
        return;
    }
    const long double c = 2.0L * xi + eta - 1.0L, t = 1.0L - eta, y = 2.0L * eta - 1.0L;
    long double q0 = 1.0L, q1 = c;  // P_a(c / t) t^a
    int idx = 0;
    for (int a = 0; a < p; ++a) {
        const long double qa = a == 0 ? q0 : q1;
        const long double al = 2 * a + 1;
        long double j0 = 1.0L, j1 = ((al + 2.0L) * y + al) / 2.0L;
        for (int b = 0; b < p - a; ++b) {
            long double jb;
            if (b == 0) jb = j0;
            else if (b == 1) jb = j1;
            else {
                const long double n = b - 1;
                const long double jn = ((2 * n + al + 1) * ((2 * n + al + 2) * (2 * n + al) * y + al * al) * j1 -
                                        2 * n * (n + al) * (2 * n + al + 2) * j0) /
                                       (2 * (n + 1) * (n + al + 1) * (2 * n + al));
                j0 = j1;
                j1 = jn;
                jb = jn;
            }
            out[idx++] = qa * jb;
        }
        if (a >= 1) {
            const long double qn = ((2 * a + 1) * c * q1 - a * t * t * q0) / (a + 1);
            q0 = q1;
            q1 = qn;
        }
    }
}

// Gauss-Jordan inverse with partial pivoting (long double); false if singular
bool invert(int n, std::vector<long double> &M, std::vector<long double> &inv) {
    inv.assign((size_t)n * n, 0.0L);
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0L;
    long double big = 0.0L;
    for (long double v : M) big = std::fmax(big, std::fabs(v));
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(M[(size_t)r * n + c]) > std::fabs(M[(size_t)piv * n + c])) piv = r;
        if (!(std::fabs(M[(size_t)piv * n + c]) > 1e-13L * big)) return false;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(M[(size_t)c * n + k], M[(size_t)piv * n + k]);
                std::swap(inv[(size_t)c * n + k], inv[(size_t)piv * n + k]);
            }
        const long double d = M[(size_t)c * n + c];
        for (int k = 0; k < n; ++k) {
            M[(size_t)c * n + k] /= d;
            inv[(size_t)c * n + k] /= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const long double f = M[(size_t)r * n + c];
            if (f == 0.0L) continue;
            for (int k = 0; k < n; ++k) {
                M[(size_t)r * n + k] -= f * M[(size_t)c * n + k];
                inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
            }
        }
    }
    return true;
}

// Rule tables shared by every cell: u points and their two weight sets, the
// v panel points, the pattern and V^-1.
struct RuleTables {
    double u[NU], wu[NU], wlog[NU];  // int_0^1 u g du = sum wu g(u_a); int_0^1 u log u g du = sum wlog g(u_a)
    double gv[NV], gw[NV];           // Gauss-Legendre on [-1, 1]
};

void build_u_rule(RuleTables &R) {
    std::vector<long double> x, w;
    gauss_legendre(NU, x, w);
    long double u[NU];
    for (int a = 0; a < NU; ++a) {
        u[a] = 0.5L * (x[a] + 1.0L);
        R.u[a] = (double)u[a];
        R.wu[a] = (double)(0.5L * w[a] * u[a]);
    }
    // int_0^1 u log u l_a(u) du over dyadic panels [2^-(k+1), 2^-k] (24-point
    // Gauss-Legendre each; the rest below 2^-64 is under 1e-36)
    std::vector<long double> gx, gw;
    gauss_legendre(24, gx, gw);
    long double acc[NU] = {0};
    for (int k = 0; k < 64; ++k) {
        const long double hi = std::ldexp(1.0L, -k), lo = hi / 2, mid = (hi + lo) / 2, half = (hi - lo) / 2;
        for (int q = 0; q < 24; ++q) {
            const long double s = mid + half * gx[q], ws = half * gw[q] * s * std::log(s);
            for (int a = 0; a < NU; ++a) {
                long double l = 1.0L;
                for (int b = 0; b < NU; ++b)
                    if (b != a) l *= (s - u[b]) / (u[a] - u[b]);
                acc[a] += ws * l;
            }
        }
    }
    for (int a = 0; a < NU; ++a) R.wlog[a] = (double)acc[a];
    gauss_legendre(NV, x, w);
    for (int b = 0; b < NV; ++b) {
        R.gv[b] = (double)x[b];
        R.gw[b] = (double)w[b];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// device
// ---------------------------------------------------------------------------
struct CorrGenArgs {
    const double *maps;   // [ncell][6]
    int64_t ncell;
    const double *ref;    // [N][2]
    const double *wref;   // [N]
    const double *vinv;   // [N][N]: (V^-1)_nj at n * N + j
    double *out;          // [ncell][N][N]
    RuleTables R;
};

template <int SHAPE, int P>
struct CellBasis;

// box: Legendre products, N = P^2
template <int P>
struct CellBasis<0, P> {
    static constexpr int N = P * P, SIDES = 4;
    static __device__ inline void corner(int k, double &x, double &y) {
        x = (k == 1 || k == 2) ? 1.0 : -1.0;
        y = (k >= 2) ? 1.0 : -1.0;
    }
    static __device__ inline void add(double xi, double eta, double c, double (&acc)[N]) {
        double lx[P], ly[P];
        lx[0] = ly[0] = 1.0;
        if (P > 1) {
            lx[1] = xi;
            ly[1] = eta;
        }
#pragma unroll
        for (int k = 2; k < P; ++k) {
            lx[k] = ((2 * k - 1) * xi * lx[k - 1] - (k - 1) * lx[k - 2]) * (1.0 / k);
            ly[k] = ((2 * k - 1) * eta * ly[k - 1] - (k - 1) * ly[k - 2]) * (1.0 / k);
        }
#pragma unroll
        for (int a = 0; a < P; ++a) {
            const double ca = c * lx[a];
#pragma unroll
            for (int b = 0; b < P; ++b) acc[a * P + b] = fma(ca, ly[b], acc[a * P + b]);
        }
    }
};

// triangle: P_a(c / t) t^a P_b^(2a+1,0)(y), a + b < P, N = P (P + 1) / 2
template <int P>
struct CellBasis<1, P> {
    static constexpr int N = P * (P + 1) / 2, SIDES = 3;
    static __device__ inline void corner(int k, double &x, double &y) {
        x = k == 1 ? 1.0 : 0.0;
        y = k == 2 ? 1.0 : 0.0;
    }
    static __device__ inline void add(double xi, double eta, double cw, double (&acc)[N]) {
        const double c = 2.0 * xi + eta - 1.0, t = 1.0 - eta, y = 2.0 * eta - 1.0;
        double q0 = 1.0, q1 = c;
        int idx = 0;
#pragma unroll
        for (int a = 0; a < P; ++a) {
            const double qa = cw * (a == 0 ? q0 : q1);
            const double al = 2 * a + 1;
            double j0 = 1.0, j1 = 0.5 * ((al + 2.0) * y + al);
#pragma unroll
            for (int b = 0; b < P - a; ++b) {
                double jb;
                if (b == 0) jb = j0;
                else if (b == 1) jb = j1;
                else {
                    const double n = b - 1;
                    const double num1 = (2 * n + al + 1) * ((2 * n + al + 2) * (2 * n + al) * y + al * al);
                    const double num0 = 2 * n * (n + al) * (2 * n + al + 2);
                    const double den = 1.0 / (2 * (n + 1) * (n + al + 1) * (2 * n + al));
                    const double jn = (num1 * j1 - num0 * j0) * den;
                    j0 = j1;
                    j1 = jn;
                    jb = jn;
                }
                acc[idx] = fma(qa, jb, acc[idx]);
                ++idx;
            }
            if (a >= 1) {
                const double qn = ((2 * a + 1) * c * q1 - a * t * t * q0) * (1.0 / (a + 1));
                q0 = q1;
                q1 = qn;
            }
        }
    }
};

// One wave per (cell, target node): the singular integrals of the basis
// (rays shared among the lanes, then summed across the wave), row i of the
// block as those integrals times V^-1 (lane j: column j), less the smooth
// terms.
template <int SHAPE, int P>
__global__ void __launch_bounds__(64) k_corr_gen(CorrGenArgs a) {
    typedef CellBasis<SHAPE, P> B;
    constexpr int N = B::N;
    static_assert(N <= 64, "one lane per column");
    const int64_t k = blockIdx.x / N;
    const int i = blockIdx.x % N;
    const int lane = threadIdx.x;
    const double *mp = a.maps + k * 6;
    const double ox = mp[0], oy = mp[1], a00 = mp[2], a01 = mp[3], a10 = mp[4], a11 = mp[5];
    const double J = fabs(a00 * a11 - a01 * a10);
    const double zx = a.ref[2 * i], zy = a.ref[2 * i + 1];
    double acc[N];
#pragma unroll
    for (int n = 0; n < N; ++n) acc[n] = 0.0;
    for (int s = 0; s < B::SIDES; ++s) {
        double px, py, qx, qy;
        B::corner(s, px, py);
        B::corner((s + 1) % B::SIDES, qx, qy);
        const double d0x = px - zx, d0y = py - zy, d1x = qx - px, d1y = qy - py;
        const double cref = fabs(d0x * d1y - d0y * d1x);
        // physical directions: A d0, A d1; nearest point of the edge at v*,
        // at distance delta (in units of the edge) from the real axis
        const double D0x = a00 * d0x + a01 * d0y, D0y = a10 * d0x + a11 * d0y;
        const double D1x = a00 * d1x + a01 * d1y, D1y = a10 * d1x + a11 * d1y;
        const double l1 = D1x * D1x + D1y * D1y;
        const double vs = -(D0x * D1x + D0y * D1y) / l1;
        const double del = fabs(D0x * D1y - D0y * D1x) / l1;
        const double vc = fmin(1.0, fmax(0.0, vs));
        const double w0 = fmax(0.5 * hypot(vs - vc, del), 1e-30);  // half-width of the first panel
        // panels: [vc - w0, vc + w0], then [vc + w0 2^m, vc + w0 2^(m+1)] and
        // mirrored, each clipped to [0, 1]
        const int nr = vc + w0 < 1.0 ? (int)ceil(log2((1.0 - vc) / w0)) : 0;
        const int nl = vc - w0 > 0.0 ? (int)ceil(log2(vc / w0)) : 0;
        const int nray = (1 + nr + nl) * NV;
        for (int r = lane; r < nray; r += 64) {
            const int pan = r / NV, b = r - pan * NV;
            double lo, hi;
            if (pan == 0) {
                lo = vc - w0;
                hi = vc + w0;
            } else if (pan <= nr) {
                lo = vc + ldexp(w0, pan - 1);
                hi = vc + ldexp(w0, pan);
            } else {
                hi = vc - ldexp(w0, pan - nr - 1);
                lo = vc - ldexp(w0, pan - nr);
            }
            lo = fmax(lo, 0.0);
            hi = fmin(hi, 1.0);
            const double half = 0.5 * (hi - lo);
            const double v = 0.5 * (hi + lo) + half * a.R.gv[b];
            const double wv = half * a.R.gw[b] * cref;
            const double ex = D0x + v * D1x, ey = D0y + v * D1y;
            const double lam = 0.5 * log(ex * ex + ey * ey);  // log|A d(v)|
            const double dx = d0x + v * d1x, dy = d0y + v * d1y;
#pragma unroll 1
            for (int q = 0; q < NU; ++q) {
                const double u = a.R.u[q];
                B::add(zx + u * dx, zy + u * dy, wv * (a.R.wlog[q] + lam * a.R.wu[q]), acc);
            }
        }
    }
    // sum over the wave, every lane keeping the total
#pragma unroll
    for (int n = 0; n < N; ++n) {
        double v = acc[n];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        acc[n] = v;
    }
    if (lane >= N) return;
    const int j = lane;
    double s = 0.0;
#pragma unroll
    for (int n = 0; n < N; ++n) s = fma(acc[n], a.vinv[n * N + j], s);
    s *= -J * INV_2PI;
    if (j != i) {
        const double rx = a.ref[2 * j] - zx, ry = a.ref[2 * j + 1] - zy;
        const double px = a00 * rx + a01 * ry, py = a10 * rx + a11 * ry;
        s -= -INV_2PI * 0.5 * log(px * px + py * py) * J * a.wref[j];
    }
    a.out[(k * N + i) * N + j] = s;
}

template <int SHAPE>
static void launch_corr_gen(int p, const CorrGenArgs &a, unsigned blocks, hipStream_t s) {
#define VP_CG(PP)                                                                                          \
    case PP:                                                                                               \
        hipLaunchKernelGGL((k_corr_gen<SHAPE, PP>), dim3(blocks), dim3(64), 0, s, a);                      \
        break;
    switch (p) {
        VP_CG(1) VP_CG(2) VP_CG(3) VP_CG(4) VP_CG(5) VP_CG(6) VP_CG(7) VP_CG(8)
        case 9:
        case 10:
            if constexpr (SHAPE == 1) {
                if (p == 9) hipLaunchKernelGGL((k_corr_gen<1, 9>), dim3(blocks), dim3(64), 0, s, a);
                else hipLaunchKernelGGL((k_corr_gen<1, 10>), dim3(blocks), dim3(64), 0, s, a);
                break;
            }
            [[fallthrough]];
        default: throw Error(VP_EUNSUPPORTED, "unsupported order");
    }
#undef VP_CG
    VP_LAUNCH_CHECK();
}

void correction_blocks(int shape, int p, const double *ref_x, const double *ref_y, const double *wref,
                       int64_t ncell, const double *maps, double *out, hipStream_t stream) {
    if (shape != VP_CELL_BOX && shape != VP_CELL_TRIANGLE) throw Error(VP_EINVAL, "unknown cell shape");
    if (p < 1) throw Error(VP_EINVAL, "order must be >= 1");
    if ((shape == VP_CELL_BOX && p > 8) || (shape == VP_CELL_TRIANGLE && p > 10))
        throw Error(VP_EUNSUPPORTED, "order above 8 (boxes) or 10 (triangles)");
    if (!ref_x || !ref_y || !wref) throw Error(VP_EINVAL, "ref_x, ref_y and wref must not be NULL");
    if (ncell < 0) throw Error(VP_EINVAL, "ncell must be >= 0");
    if (ncell > 0 && (!maps || !out)) throw Error(VP_EINVAL, "maps and out must not be NULL");
    const int N = shape == VP_CELL_BOX ? p * p : p * (p + 1) / 2;
    if (ncell * N > (int64_t)INT32_MAX) throw Error(VP_EINVAL, "too many cells for one call");
    constexpr long double MARGIN = 1e-9L;
    for (int j = 0; j < N; ++j) {
        const long double x = ref_x[j], y = ref_y[j];
        if (!std::isfinite((double)x) || !std::isfinite((double)y) || !std::isfinite(wref[j]))
            throw Error(VP_EINVAL, "non-finite node or weight in the pattern");
        const bool inside = shape == VP_CELL_BOX
                                ? (std::fabs(x) < 1.0L - MARGIN && std::fabs(y) < 1.0L - MARGIN)
                                : (x > MARGIN && y > MARGIN && x + y < 1.0L - MARGIN);
        if (!inside) throw Error(VP_EINVAL, "pattern node on or outside the reference cell");
    }
    // V^-1 in long double
    std::vector<long double> V((size_t)N * N), Vi, row(N);
    for (int j = 0; j < N; ++j) {
        basis_host(shape, p, ref_x[j], ref_y[j], row.data());
        for (int n = 0; n < N; ++n) V[(size_t)j * N + n] = row[n];
    }
    if (!invert(N, V, Vi)) throw Error(VP_EINVAL, "the node pattern is not unisolvent for the interpolation space");
    if (ncell == 0) return;
    // the maps: finite, invertible
    std::vector<double> hm((size_t)ncell * 6);
    VP_HIP(hipMemcpyAsync(hm.data(), maps, 8 * hm.size(), hipMemcpyDeviceToHost, stream));
    VP_HIP(hipStreamSynchronize(stream));
    for (int64_t k = 0; k < ncell; ++k) {
        const double *m = &hm[(size_t)k * 6];
        for (int q = 0; q < 6; ++q)
            if (!std::isfinite(m[q])) throw Error(VP_EINVAL, "non-finite cell map");
        const double det = m[2] * m[5] - m[3] * m[4];
        const double sc = std::fabs(m[2] * m[5]) + std::fabs(m[3] * m[4]);
        if (!(std::fabs(det) > 1e-14 * sc)) throw Error(VP_EINVAL, "singular cell map");
    }
    CorrGenArgs a;
    build_u_rule(a.R);
    std::vector<double> tab((size_t)2 * N + N + (size_t)N * N);
    for (int j = 0; j < N; ++j) {
        tab[2 * j] = ref_x[j];
        tab[2 * j + 1] = ref_y[j];
        tab[2 * N + j] = wref[j];
    }
    // (V^-1)_nj: Vi holds the inverse of V (rows j, columns n), Vi[n][j]
    for (int n = 0; n < N; ++n)
        for (int j = 0; j < N; ++j) tab[3 * N + (size_t)n * N + j] = (double)Vi[(size_t)n * N + j];
    double *dtab = nullptr;
    VP_HIP(hipMalloc(&dtab, 8 * tab.size()));
    try {
        VP_HIP(hipMemcpyAsync(dtab, tab.data(), 8 * tab.size(), hipMemcpyHostToDevice, stream));
        a.maps = maps;
        a.ncell = ncell;
        a.ref = dtab;
        a.wref = dtab + 2 * N;
        a.vinv = dtab + 3 * N;
        a.out = out;
        const unsigned blocks = (unsigned)(ncell * N);
        if (shape == VP_CELL_BOX) launch_corr_gen<0>(p, a, blocks, stream);
        else launch_corr_gen<1>(p, a, blocks, stream);
        VP_HIP(hipStreamSynchronize(stream));
    } catch (...) {
        (void)hipFree(dtab);
        throw;
    }
    VP_HIP(hipFree(dtab));
}

}  // namespace vp

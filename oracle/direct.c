/*
 * CPU oracle for the volume-potential hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests, the smoke check and the benchmark's cpu_baseline leg may load
 * this library.  It shares no code with the GPU library.
 *
 * What it computes is the plain definition, in float64, with Neumaier
 * compensated summation over sources so that its own rounding error is
 * ~1e-16 relative:
 *
 *   smooth part (Section 3.2, eq. Tk_smooth_quad: the target-independent
 *   rule whose "modified weights" J^k w_j turn the cell integrals into a
 *   point sum; Section 4.2 gives the same rule for boxes):
 *       s_b(t_i) = sum_j  G(r_j, t_i) * w_j * f_b(r_j)
 *   with the 2D Laplace Green's function of Section 2.1
 *       G(r, r0) = -(1/(2 pi)) log |r - r0|.
 *   A pair at exactly zero distance (the self pair when targets are the
 *   nodes) contributes nothing.
 *
 *   correction part (Section 4, the sparse matrix assembled from the local
 *   maps Pi_k next to eqs. ndofs/nsrcs):
 *       c_b(t_i) = sum_k C[i,k] f_b(r_k).
 *
 * Adjoint (exact transpose of the map f -> s + c):
 *       d_b(r_j) = w_j sum_i G(r_j, t_i) g_b(t_i) + sum_i C[i,j] g_b(t_i).
 * Target gradient of the smooth part:
 *       grad_t s_b(t) = sum_j w_j f_b(r_j) (1/(2 pi)) (r_j - t) / |r_j - t|^2.
 *
 * Arrays are C-contiguous float64; batched arrays are [nbatch][len].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_INV_2PI 0.15915494309189533576888376337251436

/* Neumaier compensated accumulator. */
typedef struct {
    double s, c;
} acc_t;

static inline void acc_add(acc_t *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static inline double acc_get(const acc_t *a) { return a->s + a->c; }

/* G(r_j, t) = -(1/2pi) log|r_j - t|; zero distance -> 0 (excluded pair). */
static inline double green(double xj, double yj, double tx, double ty) {
    double d = hypot(xj - tx, yj - ty);
    if (d == 0.0) return 0.0;
    return -ORACLE_INV_2PI * log(d);
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Smooth part at a subset of targets.
 *   n sources (x, y, w), densities f[nbatch][n]
 *   m targets (tx, ty); tidx[mt] selects the targets evaluated
 *   (tidx == NULL: all m, mt = m)
 *   out[nbatch][mt]
 */
void oracle_smooth(int64_t n, const double *x, const double *y, const double *w,
                   const double *tx, const double *ty, const int64_t *tidx, int64_t mt,
                   int nbatch, const double *f, double *out) {
    int64_t k;
#pragma omp parallel for schedule(dynamic, 16)
    for (k = 0; k < mt; ++k) {
        int64_t i = tidx ? tidx[k] : k;
        double px = tx[i], py = ty[i];
        acc_t accs[64];
        acc_t *a = accs;
        acc_t *heap = NULL;
        if (nbatch > 64) {
            heap = (acc_t *)calloc((size_t)nbatch, sizeof(acc_t));
            a = heap;
        } else {
            memset(accs, 0, sizeof(accs));
        }
        for (int64_t j = 0; j < n; ++j) {
            double g = green(x[j], y[j], px, py);
            if (g == 0.0) continue;
            double gw = g * w[j];
            for (int b = 0; b < nbatch; ++b) acc_add(&a[b], gw * f[(int64_t)b * n + j]);
        }
        for (int b = 0; b < nbatch; ++b) out[(int64_t)b * mt + k] = acc_get(&a[b]);
        free(heap);
    }
}

/*
 * Correction part at a subset of rows: out[b][k] = sum_{q in row tidx[k]} val[q] f[b][col[q]].
 */
void oracle_csr(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                const int64_t *tidx, int64_t mt, int nbatch, const double *f, double *out) {
    int64_t k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < mt; ++k) {
        int64_t i = tidx ? tidx[k] : k;
        for (int b = 0; b < nbatch; ++b) {
            acc_t a = {0.0, 0.0};
            for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q)
                acc_add(&a, val[q] * f[(int64_t)b * n + col[q]]);
            out[(int64_t)b * mt + k] = acc_get(&a);
        }
    }
}

/*
 * Transposed smooth part at a subset of sources:
 *   out[b][k] = w_j sum_i G(r_j, t_i) g[b][i],  j = sidx[k]  (sidx NULL: all n)
 */
void oracle_smooth_adjoint(int64_t n, const double *x, const double *y, const double *w,
                           int64_t m, const double *tx, const double *ty,
                           const int64_t *sidx, int64_t ns, int nbatch, const double *g,
                           double *out) {
    int64_t k;
#pragma omp parallel for schedule(dynamic, 16)
    for (k = 0; k < ns; ++k) {
        int64_t j = sidx ? sidx[k] : k;
        double px = x[j], py = y[j];
        acc_t accs[64];
        acc_t *a = accs;
        acc_t *heap = NULL;
        if (nbatch > 64) {
            heap = (acc_t *)calloc((size_t)nbatch, sizeof(acc_t));
            a = heap;
        } else {
            memset(accs, 0, sizeof(accs));
        }
        for (int64_t i = 0; i < m; ++i) {
            double gr = green(px, py, tx[i], ty[i]);
            if (gr == 0.0) continue;
            for (int b = 0; b < nbatch; ++b) acc_add(&a[b], gr * g[(int64_t)b * m + i]);
        }
        for (int b = 0; b < nbatch; ++b) out[(int64_t)b * ns + k] = w[j] * acc_get(&a[b]);
        free(heap);
    }
}

/*
 * Transposed correction part at a subset of columns:
 *   out[b][k] = sum_i C[i, j] g[b][i],  j = sidx[k].
 * A plain scan over all nonzeros (serial, no races), then a pick.
 */
void oracle_csr_adjoint(int64_t n, int64_t m, const int64_t *rowptr, const int32_t *col,
                        const double *val, const int64_t *sidx, int64_t ns, int nbatch,
                        const double *g, double *out) {
    acc_t *full = (acc_t *)calloc((size_t)n * (size_t)nbatch, sizeof(acc_t));
    for (int64_t i = 0; i < m; ++i)
        for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q)
            for (int b = 0; b < nbatch; ++b)
                acc_add(&full[(int64_t)b * n + col[q]], val[q] * g[(int64_t)b * m + i]);
    for (int64_t k = 0; k < ns; ++k) {
        int64_t j = sidx ? sidx[k] : k;
        for (int b = 0; b < nbatch; ++b) out[(int64_t)b * ns + k] = acc_get(&full[(int64_t)b * n + j]);
    }
    free(full);
}

/*
 * Gradient of the smooth part with respect to the target position:
 *   out[b][0][k], out[b][1][k]  (d/dtx, d/dty) at target tidx[k].
 */
void oracle_smooth_grad(int64_t n, const double *x, const double *y, const double *w,
                        const double *tx, const double *ty, const int64_t *tidx, int64_t mt,
                        int nbatch, const double *f, double *out) {
    int64_t k;
#pragma omp parallel for schedule(dynamic, 16)
    for (k = 0; k < mt; ++k) {
        int64_t i = tidx ? tidx[k] : k;
        double px = tx[i], py = ty[i];
        acc_t ax[64], ay[64];
        acc_t *gx = ax, *gy = ay, *heap = NULL;
        if (nbatch > 64) {
            heap = (acc_t *)calloc(2 * (size_t)nbatch, sizeof(acc_t));
            gx = heap;
            gy = heap + nbatch;
        } else {
            memset(ax, 0, sizeof(ax));
            memset(ay, 0, sizeof(ay));
        }
        for (int64_t j = 0; j < n; ++j) {
            double dx = x[j] - px, dy = y[j] - py;
            double d2 = dx * dx + dy * dy;
            if (d2 == 0.0) continue;
            double s = ORACLE_INV_2PI * w[j] / d2;
            for (int b = 0; b < nbatch; ++b) {
                double q = f[(int64_t)b * n + j] * s;
                acc_add(&gx[b], q * dx);
                acc_add(&gy[b], q * dy);
            }
        }
        for (int b = 0; b < nbatch; ++b) {
            out[((int64_t)b * 2 + 0) * mt + k] = acc_get(&gx[b]);
            out[((int64_t)b * 2 + 1) * mt + k] = acc_get(&gy[b]);
        }
        free(heap);
    }
}

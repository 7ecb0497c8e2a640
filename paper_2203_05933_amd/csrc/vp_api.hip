// C ABI of libvp (declared in include/vp.h): argument validation, plan
// construction and the evaluation entry points.  Internal errors are C++
// exceptions, caught here and turned into vp_status codes.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "vp_internal.hpp"

namespace vp {

// The two auxiliary streams are shared by every plan on a device (created
// with the first plan, destroyed with the last): each stream takes a
// hardware queue, and a process has few (GPU_MAX_HW_QUEUES, 4 by default);
// streams beyond that share queues and serialise kernels that were meant to
// overlap.  Sharing only adds ordering: every cross-stream wait of an
// evaluation is on an event recorded before the wait, so concurrent plans
// cannot deadlock.
struct SharedStreams {
    hipStream_t aux = nullptr, aux2 = nullptr;
    int refs = 0;
};
static std::mutex g_streams_mu;
static std::map<int, SharedStreams> g_streams;

static void acquire_streams(vp_plan_s *P) {
    std::lock_guard<std::mutex> lk(g_streams_mu);
    SharedStreams &S = g_streams[P->device];
    if (S.refs == 0) {
        VP_HIP(hipStreamCreateWithFlags(&S.aux, hipStreamNonBlocking));
        hipError_t e = hipStreamCreateWithFlags(&S.aux2, hipStreamNonBlocking);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(S.aux);
            S.aux = nullptr;
            VP_HIP(e);
        }
    }
    ++S.refs;
    P->aux = S.aux;
    P->aux2 = S.aux2;
}

static void release_streams(vp_plan_s *P) {
    if (!P->aux) return;
    std::lock_guard<std::mutex> lk(g_streams_mu);
    SharedStreams &S = g_streams[P->device];
    (void)hipStreamSynchronize(P->aux);
    (void)hipStreamSynchronize(P->aux2);
    P->aux = P->aux2 = nullptr;
    if (--S.refs == 0) {
        (void)hipStreamDestroy(S.aux);
        (void)hipStreamDestroy(S.aux2);
        S.aux = S.aux2 = nullptr;
    }
}

[[noreturn]] void throw_hip(hipError_t e, const char *expr, const char *file, int line) {
    char buf[512];
    std::snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), expr,
                  file, line);
    throw Error(VP_EDEVICE, buf);
}

// ---------------------------------------------------------------------------
// Static evaluation workspace (vp_eval_noalloc).  Each device that loads the
// library's code object holds its own copy of `scratch` until the process
// ends.  In host code the array's name is not a device address: its address
// on a device comes from hipGetSymbolAddress, resolved once per device with
// that device current (at plan time) and kept in g_scratch; host code passes
// only that address on.
// ---------------------------------------------------------------------------
__device__ __align__(256) unsigned char scratch[VP_NOALLOC_MAX_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch;

// address of this device's scratch array; the device must be current
static void *scratch_address(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(device);
    if (it != g_scratch.end()) return it->second;
    void *ptr = nullptr;
    VP_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw Error(VP_EDEVICE, "hipGetSymbolAddress returned no address for the static workspace");
    g_scratch[device] = ptr;
    return ptr;
}

// The evaluation workspace carved from one base address, each part aligned
// to 256 bytes; returns the bytes used (base == nullptr: only the size).
static size_t carve_workspace(vp_plan_s *P, unsigned char *base, double **q, double **acc, double **acc_far,
                              void **M, void **L, double **qi) {
    const int64_t len = std::max(P->n, P->m);
    const size_t esz = P->fp32 ? 4 : 8;
    const size_t ecount = (size_t)P->tree.nbox * P->nbatch * P->PD;
    const size_t mcount = (size_t)P->mexp_boxes() * P->nbatch * P->PD;
    const size_t sizes[6] = {8 * (size_t)P->nbatch * len, 8 * (size_t)P->nbatch * len,
                             8 * (size_t)P->nbatch * len, mcount * esz,
                             ecount * esz,                 P->qi ? 8 * (size_t)P->nbatch * (len + QI_ZERO_PTS) : 0};
    void *parts[6];
    size_t off = 0;
    for (int k = 0; k < 6; ++k) {
        parts[k] = base ? base + off : nullptr;
        off += (sizes[k] + 255) / 256 * 256;
    }
    if (base) {
        *q = static_cast<double *>(parts[0]);
        *acc = static_cast<double *>(parts[1]);
        *acc_far = static_cast<double *>(parts[2]);
        *M = parts[3];
        *L = parts[4];
        if (P->qi) *qi = static_cast<double *>(parts[5]);
    }
    return off;
}

}  // namespace vp

using vp::Error;

// ---------------------------------------------------------------------------
// per-stage timing
// ---------------------------------------------------------------------------
void vp_plan_s::timing_eval_begin() {
    if (!timing) return;
    if (tcount - tdone >= TRING) timing_collect(tcount - TRING + 1);
    tcur = (int)(tcount % TRING);
    tslot_used[tcur] = 0;
    ++tcount;
}
void vp_plan_s::stage_begin(int st) {
    if (!timing || tcur < 0) return;
    VP_HIP(hipEventRecord(tev[((size_t)tcur * VP_NSTAGES + st) * 2], stream));
    tslot_used[tcur] |= 1 << st;
}
void vp_plan_s::stage_end(int st) {
    if (!timing || tcur < 0) return;
    VP_HIP(hipEventRecord(tev[((size_t)tcur * VP_NSTAGES + st) * 2 + 1], stream));
}
void vp_plan_s::timing_collect(int64_t upto) {
    for (; tdone < upto; ++tdone) {
        int slot = (int)(tdone % TRING);
        for (int st = 0; st < VP_NSTAGES; ++st) {
            if (!(tslot_used[slot] & (1 << st))) continue;
            hipEvent_t a = tev[((size_t)slot * VP_NSTAGES + st) * 2], b = tev[((size_t)slot * VP_NSTAGES + st) * 2 + 1];
            VP_HIP(hipEventSynchronize(b));
            float ms = 0.f;
            VP_HIP(hipEventElapsedTime(&ms, a, b));
            tms[st] += ms;
        }
    }
}

static thread_local std::string g_last_error;

static vp_status set_err(vp_plan_s *P, vp_status st, const std::string &msg) {
    if (P) {
        P->err = msg;
        if (st == VP_EDEVICE) P->poisoned = true;
    } else {
        g_last_error = msg;
    }
    return st;
}

template <class F>
static vp_status guarded(vp_plan_s *P, F &&fn) {
    try {
        fn();
        return VP_OK;
    } catch (const Error &e) {
        return set_err(P, e.status, e.what());
    } catch (const std::bad_alloc &) {
        return set_err(P, VP_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return set_err(P, VP_EINTERNAL, e.what());
    } catch (...) {
        return set_err(P, VP_EINTERNAL, "unknown internal error");
    }
}

extern "C" void vp_default_options(vp_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->order = 30;
    opt->max_leaf = 64;
    opt->nbatch = 1;
    opt->precision = VP_FP64;
    opt->m2l_mode = VP_M2L_AUTO;
    opt->p2p_mode = VP_P2P_AUTO;
    opt->max_level = 0;
    opt->flags = 0;
    opt->root[0] = opt->root[1] = opt->root[2] = 0.0;
    opt->stream = nullptr;
    opt->kernel = VP_KERNEL_LAPLACE;
    opt->lambda = 0.0;
}

static void validate_plan_args(const double *x, const double *y, const double *w, int64_t n,
                               const double *tx, const double *ty, int64_t m, const int64_t *rowptr,
                               const int32_t *col, const double *val, const vp_options &o,
                               vp_plan_t *out, int64_t nd) {
    auto bad = [](const std::string &s) { throw Error(VP_EINVAL, s); };
    if (!out) bad("out is NULL");
    if (!x || !y || !w) bad("x, y and w must not be NULL");
    if (n < 1) bad("n must be >= 1");
    if (n > 0x3FFFFFFF) bad("n too large (must fit 30-bit indices)");
    if ((tx == nullptr) != (ty == nullptr)) bad("tx and ty must both be NULL or both non-NULL");
    if (!tx && m != n) bad("targets are the nodes (tx == ty == NULL) but m != n");
    if (m < 1) bad("m must be >= 1");
    if (m > 0x3FFFFFFF) bad("m too large");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i]) || !std::isfinite(y[i]) || !std::isfinite(w[i]))
            bad("non-finite node coordinate or weight at index " + std::to_string(i));
    if (tx)
        for (int64_t i = 0; i < m; ++i)
            if (!std::isfinite(tx[i]) || !std::isfinite(ty[i]))
                bad("non-finite target coordinate at index " + std::to_string(i));
    if (rowptr) {
        if (!col && rowptr[m] > 0) bad("col is NULL");
        if (!val && rowptr[m] > 0) bad("val is NULL");
        if (rowptr[0] != 0) bad("rowptr[0] must be 0");
        for (int64_t i = 0; i < m; ++i)
            if (rowptr[i + 1] < rowptr[i]) bad("rowptr must be non-decreasing (row " + std::to_string(i) + ")");
        int64_t nnz = rowptr[m];
        if (nnz > 0x7FFFFFFF) throw Error(VP_EUNSUPPORTED, "more than 2^31-1 correction non-zeros");
        for (int64_t q = 0; q < nnz; ++q)
            if (col[q] < 0 || col[q] >= nd) bad("col out of range at non-zero " + std::to_string(q));
        for (int64_t q = 0; q < nnz; ++q)
            if (!std::isfinite(val[q])) bad("non-finite correction value at non-zero " + std::to_string(q));
    }
    if (o.order < 1 || o.order > 60) bad("order must be in 1..60");
    if (o.max_leaf < 1 || o.max_leaf > 256) bad("max_leaf must be in 1..256");
    if (o.nbatch < 1 || o.nbatch > vp::MAX_BATCH) bad("nbatch must be in 1..64");
    if (o.precision != VP_FP64 && o.precision != VP_FP32_BULK) bad("unknown precision");
    if (o.m2l_mode < 0 || o.m2l_mode > 5) bad("unknown m2l_mode");
    if (o.precision == VP_FP64 && (o.m2l_mode == VP_M2L_FP32_MFMA || o.m2l_mode == VP_M2L_FP32_SPLIT ||
                                   o.m2l_mode == VP_M2L_FP32_SCALED))
        bad("FP32 M2L modes need precision VP_FP32_BULK");
    if (o.p2p_mode < 0 || o.p2p_mode > 2) bad("unknown p2p_mode");
    if (o.max_level < 0 || o.max_level > vp::LBITS) bad("max_level must be in 0..30");
    if (o.flags & ~(VP_FLAG_AUTOTUNE | VP_FLAG_ONE_STREAM | VP_FLAG_AUTOTUNE_LEAF)) bad("unknown flags");
    if (o.kernel != VP_KERNEL_LAPLACE && o.kernel != VP_KERNEL_YUKAWA) bad("unknown kernel");
    if (o.m2l_waves != 0 && o.m2l_waves != 1 && o.m2l_waves != 2 && o.m2l_waves != 4)
        bad("m2l_waves must be 0, 1, 2 or 4");
    if (o.table_waves != 0 && o.table_waves != 1 && o.table_waves != 2 && o.table_waves != 4)
        bad("table_waves must be 0, 1, 2 or 4");
    if (o.kernel == VP_KERNEL_YUKAWA && !(std::isfinite(o.lambda) && o.lambda > 0))
        bad("the modified Helmholtz kernel needs a finite lambda > 0");
    if (o.kernel == VP_KERNEL_YUKAWA && o.precision != VP_FP64)
        throw Error(VP_EUNSUPPORTED, "the modified Helmholtz kernel runs in float64 only");
    if (o.kernel == VP_KERNEL_YUKAWA && o.p2p_mode == VP_P2P_PAIRWISE)
        throw Error(VP_EUNSUPPORTED, "the modified Helmholtz kernel has no pairwise near-field kernel");
    if (o.root[2] > 0 && (!std::isfinite(o.root[0]) || !std::isfinite(o.root[1]) || !std::isfinite(o.root[2])))
        bad("non-finite root square");
    if (o.root[2] > 0) {
        // every node and target must lie in the closed root square: a point
        // outside would be quantised into a border box whose expansion centre
        // it is not near, and the far field would lose its accuracy silently
        const double x0 = o.root[0], y0 = o.root[1], x1 = o.root[0] + o.root[2], y1 = o.root[1] + o.root[2];
        auto outside = [&](double px, double py) { return px < x0 || px > x1 || py < y0 || py > y1; };
        for (int64_t i = 0; i < n; ++i)
            if (outside(x[i], y[i])) bad("node " + std::to_string(i) + " lies outside the root square");
        if (tx)
            for (int64_t i = 0; i < m; ++i)
                if (outside(tx[i], ty[i])) bad("target " + std::to_string(i) + " lies outside the root square");
    }
}

static void release_timing(vp_plan_s *P) {
    for (hipEvent_t e : P->tev) (void)hipEventDestroy(e);
    P->tev.clear();
    P->timing = false;
}

static void free_plan(vp_plan_s *P) {
    if (!P) return;
    if (P->stream) (void)hipStreamSynchronize(P->stream);
    else (void)hipDeviceSynchronize();
    vp::release_streams(P);
    for (hipEvent_t e : {P->ev_fork, P->ev_join, P->ev_p2m, P->ev_p2l, P->ev_upper, P->ev_coarse, P->ev_m2p})
        if (e) (void)hipEventDestroy(e);
    release_timing(P);
    P->mem.free_all();
    delete P;
}

// ---------------------------------------------------------------------------
// Tuning cache: the autotuner's choices per geometry and options, for the
// life of the process
// ---------------------------------------------------------------------------
struct TuneChoice {
    int m2l_mode = 0, m2l_nw = 1, table_nw = 1, one_stream = 0, max_leaf = 0;
    float ms = 0.f;
};
static std::mutex g_tune_mu;
static std::map<std::string, TuneChoice> g_tune;

static uint64_t fnv1a(uint64_t h, const void *p, size_t bytes) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < bytes; ++i) h = (h ^ c[i]) * 1099511628211ull;
    return h;
}

// key: sizes, the options that shape the evaluation (max_leaf only when the
// leaf size is not itself tuned) and a hash of the coordinates
static std::string tune_key(const double *x, const double *y, int64_t n, const double *tx, const double *ty,
                            int64_t m, int64_t nnz, const vp_oversampling *os, const vp_options &o) {
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(h, x, 8 * (size_t)n);
    h = fnv1a(h, y, 8 * (size_t)n);
    if (tx) {
        h = fnv1a(h, tx, 8 * (size_t)m);
        h = fnv1a(h, ty, 8 * (size_t)m);
    }
    char buf[512];
    std::snprintf(buf, sizeof(buf), "%lld/%lld/%lld/%d/%d/%d/%d/%d/%d/%d/%d/%.17g/%.17g/%.17g/%.17g/%d/%d/%d/%d/%llx",
                  (long long)n, (long long)m, (long long)nnz, o.order,
                  (o.flags & VP_FLAG_AUTOTUNE_LEAF) ? -1 : o.max_leaf, o.nbatch, o.precision, o.p2p_mode,
                  o.max_level, o.kernel, (o.flags & (VP_FLAG_ONE_STREAM | VP_FLAG_AUTOTUNE_LEAF)), o.root[0],
                  o.root[1], o.root[2], o.lambda, os ? os->p : 0, os ? os->q : 0, o.m2l_waves, o.table_waves,
                  (unsigned long long)h);
    return buf;
}

static bool tune_lookup(const std::string &key, TuneChoice &c) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    c = it->second;
    return true;
}

static void tune_store(const std::string &key, const TuneChoice &c) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = c;
}

// Oversampled boxes: checks of the layout (see vp_plan_oversampled)
static void validate_oversampling(const vp_oversampling *os, int64_t n, const double *tx) {
    auto bad = [](const std::string &s) { throw Error(VP_EINVAL, s); };
    if (!tx) bad("an oversampled plan needs its targets (tx, ty): the density nodes are not the sources");
    if (os->p < 1 || os->q < os->p || os->q > 32) bad("oversampling needs 1 <= p <= q <= 32");
    if (os->nbox < 1) bad("oversampling needs at least one box");
    if (!os->in_start || !os->out_start) bad("in_start and out_start must not be NULL");
    if (os->n_in < 1 || os->n_in > 0x3FFFFFFF) bad("n_in must be in 1..2^30-1");
    const int64_t p2 = (int64_t)os->p * os->p, q2 = (int64_t)os->q * os->q;
    if (os->nbox * q2 != n) bad("the boxes' q x q source blocks must cover the n sources exactly");
    std::vector<std::pair<int64_t, int64_t>> in(os->nbox), outr(os->nbox);
    for (int64_t b = 0; b < os->nbox; ++b) {
        if (os->in_start[b] < 0 || os->in_start[b] + p2 > os->n_in)
            bad("box " + std::to_string(b) + ": density values out of range");
        if (os->out_start[b] < 0 || os->out_start[b] + q2 > n)
            bad("box " + std::to_string(b) + ": source nodes out of range");
        in[b] = {os->in_start[b], b};
        outr[b] = {os->out_start[b], b};
    }
    std::sort(in.begin(), in.end());
    std::sort(outr.begin(), outr.end());
    for (int64_t b = 1; b < os->nbox; ++b) {
        if (in[b].first < in[b - 1].first + p2) bad("the boxes' density values overlap");
        if (outr[b].first < outr[b - 1].first + q2) bad("the boxes' source nodes overlap");
    }
}

// 1D map from the values at the p roots of T_p (ascending) to the degree
// < p interpolant's values at the q roots of T_q, by the barycentric formula
// with the weights of Chebyshev points of the first kind,
// lambda_i = (-1)^i sin((2i+1) pi / 2p) (a common sign cancels); rows [q][p].
static std::vector<long double> cheb_interp_1d(int p, int q) {
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<long double> xp(p), xq(q), lam(p), L((size_t)q * p, 0.0L);
    for (int i = 0; i < p; ++i) {
        xp[i] = -std::cos((2 * i + 1) * pi / (2 * p));
        lam[i] = ((i & 1) ? -1.0L : 1.0L) * std::sin((2 * i + 1) * pi / (2 * p));
    }
    for (int j = 0; j < q; ++j) xq[j] = -std::cos((2 * j + 1) * pi / (2 * q));
    for (int j = 0; j < q; ++j) {
        int hit = -1;
        for (int i = 0; i < p; ++i)
            if (xq[j] == xp[i]) hit = i;
        if (hit >= 0) {
            L[(size_t)j * p + hit] = 1.0L;
            continue;
        }
        long double den = 0.0L;
        for (int i = 0; i < p; ++i) den += lam[i] / (xq[j] - xp[i]);
        for (int i = 0; i < p; ++i) L[(size_t)j * p + i] = lam[i] / (xq[j] - xp[i]) / den;
    }
    return L;
}

static void build_oversampling(vp_plan_s *P, const vp_oversampling *os) {
    const int p = os->p, q = os->q, p2 = p * p, q2 = q * q;
    P->os_p = p;
    P->os_q = q;
    P->os_nbox = os->nbox;
    const std::vector<long double> L = cheb_interp_1d(p, q);
    // tensor product, node a = jy * n + jx on both sides
    std::vector<double> O((size_t)q2 * p2), OT((size_t)p2 * q2);
    for (int jy = 0; jy < q; ++jy)
        for (int jx = 0; jx < q; ++jx)
            for (int iy = 0; iy < p; ++iy)
                for (int ix = 0; ix < p; ++ix) {
                    const double v = (double)(L[(size_t)jy * p + iy] * L[(size_t)jx * p + ix]);
                    const int r = jy * q + jx, c = iy * p + ix;
                    O[(size_t)r * p2 + c] = v;
                    OT[(size_t)c * q2 + r] = v;
                }
    P->os_O = P->mem.alloc<double>(O.size());
    P->os_OT = P->mem.alloc<double>(OT.size());
    P->os_in = P->mem.alloc<int64_t>(os->nbox);
    P->os_out = P->mem.alloc<int64_t>(os->nbox);
    VP_HIP(hipMemcpyAsync(P->os_O, O.data(), 8 * O.size(), hipMemcpyHostToDevice, P->stream));
    VP_HIP(hipMemcpyAsync(P->os_OT, OT.data(), 8 * OT.size(), hipMemcpyHostToDevice, P->stream));
    VP_HIP(hipMemcpyAsync(P->os_in, os->in_start, 8 * os->nbox, hipMemcpyHostToDevice, P->stream));
    VP_HIP(hipMemcpyAsync(P->os_out, os->out_start, 8 * os->nbox, hipMemcpyHostToDevice, P->stream));
    VP_HIP(hipStreamSynchronize(P->stream));  // the host copies leave scope
}

static vp_status plan_build(const double *x, const double *y, const double *w, int64_t n, const double *tx,
                            const double *ty, int64_t m, const int64_t *rowptr, const int32_t *col,
                            const double *val, const vp_oversampling *os, const vp_options *opt, vp_plan_t *out) {
    if (out) *out = nullptr;
    vp_options o;
    if (opt) o = *opt;
    else vp_default_options(&o);
    vp_plan_s *P = nullptr;
    vp_status st = guarded(nullptr, [&] {
        if (os) validate_oversampling(os, n, tx);
        const int64_t nd = os ? os->n_in : n;
        validate_plan_args(x, y, w, n, tx, ty, m, rowptr, col, val, o, out, nd);
        P = new vp_plan_s();
        P->opt = o;
        P->n = n;
        P->m = m;
        P->nd = nd;
        P->self = (tx == nullptr);
        P->nbatch = o.nbatch;
        P->p = o.order;
        P->P = o.order + 1;
        // rows per expansion column: 2P values, the A_0 sum row of the
        // per-offset M2L form, zero padding to a multiple of 16, and at least
        // P + PQ rows (PQ = P rounded up to 16) so that the scaled M2L reads
        // coefficient rows k < PQ of both parts without a clamp
        {
            const int PQ = (P->P + 15) / 16 * 16;
            P->PD = (std::max(2 * P->P + 1, P->P + PQ) + 15) / 16 * 16;
        }
        if (P->PD > 128) throw Error(VP_EUNSUPPORTED, "order too large (2(p+1)+1 must be <= 128)");
        P->fp32 = (o.precision == VP_FP32_BULK);
        P->one_stream = (o.flags & VP_FLAG_ONE_STREAM) != 0;
        if (o.m2l_waves) P->m2l_nw = o.m2l_waves;
        if (o.table_waves) P->table_nw = o.table_waves;
        P->m2l_mode = o.m2l_mode == VP_M2L_AUTO ? (P->fp32 ? VP_M2L_FP32_SCALED : VP_M2L_FP64_SCALED) : o.m2l_mode;
        P->stream = static_cast<hipStream_t>(o.stream);
        VP_HIP(hipGetDevice(&P->device));
        P->scratch_dev = vp::scratch_address(P->device);
        if (os) build_oversampling(P, os);
        vp::acquire_streams(P);
        for (hipEvent_t *e : {&P->ev_fork, &P->ev_join, &P->ev_p2m, &P->ev_p2l, &P->ev_upper, &P->ev_coarse, &P->ev_m2p})
            VP_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
        P->err_flag = P->mem.alloc<int32_t>(1);
        P->w_user = P->mem.alloc<double>(n);
        VP_HIP(hipMemcpyAsync(P->w_user, w, sizeof(double) * n, hipMemcpyHostToDevice, P->stream));
        vp::build_tree(P, x, y, tx, ty);
        vp::build_operators(P);
        // correction matrix
        P->nnz = rowptr ? rowptr[m] : 0;
        P->rowptr = P->mem.alloc<int64_t>(m + 1);
        if (rowptr) {
            VP_HIP(hipMemcpyAsync(P->rowptr, rowptr, sizeof(int64_t) * (m + 1), hipMemcpyHostToDevice, P->stream));
        } else {
            std::vector<int64_t> z(m + 1, 0);
            VP_HIP(hipMemcpyAsync(P->rowptr, z.data(), sizeof(int64_t) * (m + 1), hipMemcpyHostToDevice, P->stream));
            VP_HIP(hipStreamSynchronize(P->stream));
        }
        P->col = P->mem.alloc<int32_t>(P->nnz);
        // values padded to an even count with zeros (the correction kernel reads aligned pairs)
        P->val = P->mem.alloc<double>(P->nnz + 2);
        vp::fill_f64(P->val + P->nnz, 0.0, 2, P->stream);
        if (P->nnz > 0) {
            VP_HIP(hipMemcpyAsync(P->col, col, sizeof(int32_t) * P->nnz, hipMemcpyHostToDevice, P->stream));
            VP_HIP(hipMemcpyAsync(P->val, val, sizeof(double) * P->nnz, hipMemcpyHostToDevice, P->stream));
        }
        vp::build_csr_transpose(P);
        vp::detect_runs(P);
        vp::build_schedules(P);
        // workspace
        const int64_t len = std::max(n, m);
        P->q = P->mem.alloc<double>((size_t)P->nbatch * len);
        P->acc = P->mem.alloc<double>((size_t)P->nbatch * 2 * len);
        P->acc_far = P->mem.alloc<double>((size_t)P->nbatch * len);
        const size_t esz = P->fp32 ? 4 : 8;
        // multipoles also for the virtual children of X-list sources
        const size_t ecount = (size_t)P->tree.nbox * P->nbatch * P->PD;
        const size_t mcount = (size_t)P->mexp_boxes() * P->nbatch * P->PD;
        P->Mexp = P->mem.alloc<unsigned char>(mcount * esz);
        P->Lexp = P->mem.alloc<unsigned char>(ecount * esz);
        // zeros read in place of an absent source column (M2L, near tables)
        const int64_t nzero = std::max<int64_t>(P->PD, 128 * (int64_t)P->nbatch);
        P->zero_col = P->mem.alloc<double>(nzero);
        vp::fill_f64((double *)P->zero_col, 0.0, nzero, P->stream);
        if (P->fp32) {
            vp::fill_f32((float *)P->Mexp, 0.f, (int64_t)mcount, P->stream);
            vp::fill_f32((float *)P->Lexp, 0.f, (int64_t)ecount, P->stream);
        } else {
            vp::fill_f64((double *)P->Mexp, 0.0, (int64_t)mcount, P->stream);
            vp::fill_f64((double *)P->Lexp, 0.0, (int64_t)ecount, P->stream);
        }
        VP_HIP(hipStreamSynchronize(P->stream));
        vp::build_near_tables(P);
        {
            const vp::NearTables &N = P->near;
            P->q_pattern_only = N.active && o.kernel != VP_KERNEL_YUKAWA && N.n_p2m_jobs_rest == 0 &&
                                N.n_p2m_cols == N.n_p2m_leaf_cols && P->n_x_boxes == 0 && N.n_rest_leaves == 0;
        }
        // the near tables read their source columns from a density-fastest copy
        // of the charges (one box's columns are one contiguous block)
        if (P->near.active && P->nbatch > 1) {
            P->qi = P->mem.alloc<double>((size_t)P->nbatch * (len + vp::QI_ZERO_PTS));
            P->qi_zero = len;
            vp::fill_f64(P->qi + len * P->nbatch, 0.0, (int64_t)vp::QI_ZERO_PTS * P->nbatch, P->stream);
        }
        if (o.kernel == VP_KERNEL_YUKAWA) vp::build_yukawa(P);
        if (o.p2p_mode == VP_P2P_TABLES && !P->near.active)
            throw Error(VP_EUNSUPPORTED, "p2p_mode TABLES needs targets = nodes and congruent leaves");
        if ((o.flags & VP_FLAG_AUTOTUNE) && o.m2l_mode == VP_M2L_AUTO && !P->yk.active) {
            const std::string key = tune_key(x, y, n, tx, ty, m, rowptr ? rowptr[m] : 0, os, o);
            TuneChoice c;
            if (tune_lookup(key, c)) {
                P->m2l_mode = c.m2l_mode;
                P->m2l_nw = c.m2l_nw;
                P->table_nw = c.table_nw;
                P->one_stream = c.one_stream != 0;
                P->tuned = 2;
            } else {
                const auto t0 = std::chrono::steady_clock::now();
                c.ms = vp::autotune(P);
                P->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                P->tuned = 1;
                c.m2l_mode = P->m2l_mode;
                c.m2l_nw = P->m2l_nw;
                c.table_nw = P->table_nw;
                c.one_stream = P->one_stream ? 1 : 0;
                tune_store(key, c);
            }
        }
    });
    if (st != VP_OK) {
        free_plan(P);  // the message is already in the thread-local slot
        return st;
    }
    *out = P;
    return VP_OK;
}

// Plan with VP_FLAG_AUTOTUNE_LEAF: build the plan with max_leaf and with
// max_leaf / 4, time a forward evaluation of each (density 1) and keep the
// faster; the choice is cached like the other tuned knobs.
static vp_status plan_impl(const double *x, const double *y, const double *w, int64_t n, const double *tx,
                           const double *ty, int64_t m, const int64_t *rowptr, const int32_t *col,
                           const double *val, const vp_oversampling *os, const vp_options *opt, vp_plan_t *out) {
    vp_options o;
    if (opt) o = *opt;
    else vp_default_options(&o);
    if (!(o.flags & VP_FLAG_AUTOTUNE_LEAF)) return plan_build(x, y, w, n, tx, ty, m, rowptr, col, val, os, &o, out);
    if (out) *out = nullptr;
    if (!out) return set_err(nullptr, VP_EINVAL, "out is NULL");
    vp_options base = o;
    base.flags &= ~VP_FLAG_AUTOTUNE_LEAF;
    if (o.max_leaf < 1 || o.max_leaf > 256) return plan_build(x, y, w, n, tx, ty, m, rowptr, col, val, os, &base, out);
    const std::string key = tune_key(x, y, n, tx, ty, m, rowptr ? rowptr[m] : 0, os, o);
    TuneChoice c;
    if (tune_lookup(key, c) && c.max_leaf > 0) {
        base.max_leaf = c.max_leaf;
        vp_status st = plan_build(x, y, w, n, tx, ty, m, rowptr, col, val, os, &base, out);
        if (st == VP_OK) (*out)->tuned = 2;
        return st;
    }
    std::vector<int> cand{o.max_leaf};
    if (o.max_leaf / 4 >= 4) cand.push_back(o.max_leaf / 4);
    const auto t0 = std::chrono::steady_clock::now();
    vp_plan_s *best = nullptr;
    float best_ms = 1e30f;
    vp_status last = VP_OK;
    std::string last_msg;
    for (int leaf : cand) {
        base.max_leaf = leaf;
        vp_plan_t Pc = nullptr;
        vp_status st = plan_build(x, y, w, n, tx, ty, m, rowptr, col, val, os, &base, &Pc);
        if (st != VP_OK) {
            last = st;
            last_msg = g_last_error;
            continue;
        }
        float ms = 1e30f;
        st = guarded(Pc, [&] {
            vp::TempArena tmp;
            double *f = tmp.alloc<double>((size_t)Pc->nbatch * Pc->nd);
            double *u = tmp.alloc<double>((size_t)Pc->nbatch * Pc->m);
            vp::fill_f64(f, 1.0, (int64_t)Pc->nbatch * Pc->nd, Pc->stream);
            ms = vp::time_forward(Pc, f, u, 3);
            VP_HIP(hipStreamSynchronize(Pc->stream));
        });
        if (st != VP_OK) {
            last = st;
            last_msg = Pc->err;
            free_plan(Pc);
            continue;
        }
        if (ms < best_ms) {
            if (best) free_plan(best);
            best = Pc;
            best_ms = ms;
        } else {
            free_plan(Pc);
        }
    }
    if (!best) {
        g_last_error = last_msg;
        return last == VP_OK ? VP_EINTERNAL : last;
    }
    c.max_leaf = best->opt.max_leaf;
    c.m2l_mode = best->m2l_mode;
    c.m2l_nw = best->m2l_nw;
    c.table_nw = best->table_nw;
    c.one_stream = best->one_stream ? 1 : 0;
    c.ms = best_ms;
    tune_store(key, c);
    if (!best->tuned) best->tuned = 1;
    best->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = best;
    return VP_OK;
}

extern "C" vp_status vp_plan(const double *x, const double *y, const double *w, int64_t n, const double *tx,
                             const double *ty, int64_t m, const int64_t *rowptr, const int32_t *col,
                             const double *val, const vp_options *opt, vp_plan_t *out) {
    return plan_impl(x, y, w, n, tx, ty, m, rowptr, col, val, nullptr, opt, out);
}

extern "C" vp_status vp_plan_oversampled(const double *x, const double *y, const double *w, int64_t n,
                                         const double *tx, const double *ty, int64_t m, const int64_t *rowptr,
                                         const int32_t *col, const double *val, const vp_oversampling *os,
                                         const vp_options *opt, vp_plan_t *out) {
    if (!os) {
        if (out) *out = nullptr;
        return set_err(nullptr, VP_EINVAL, "os is NULL");
    }
    return plan_impl(x, y, w, n, tx, ty, m, rowptr, col, val, os, opt, out);
}

static bool overlaps(const void *a, size_t abytes, const void *b, size_t bbytes) {
    auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + bbytes && pb < pa + abytes;
}

extern "C" vp_status vp_eval(vp_plan_t P, const double *f, double *u) {
    if (!P) return set_err(nullptr, VP_EINVAL, "plan is NULL");
    if (P->poisoned) return set_err(P, VP_EDEVICE, "plan is poisoned by an earlier device error: " + P->err);
    if (!f || !u) return set_err(P, VP_EINVAL, "f and u must not be NULL");
    if (overlaps(f, 8 * (size_t)P->nbatch * P->nd, u, 8 * (size_t)P->nbatch * P->m))
        return set_err(P, VP_EINVAL, "f and u overlap");
    return guarded(P, [&] {
        P->timing_eval_begin();
        vp::prepare_charges(P, f, false);
        vp::run_fmm(P, false, false, f, u);
    });
}

extern "C" vp_status vp_eval_noalloc(vp_plan_t P, const double *f, double *u) {
    if (!P) return set_err(nullptr, VP_EINVAL, "plan is NULL");
    if (P->poisoned) return set_err(P, VP_EDEVICE, "plan is poisoned by an earlier device error: " + P->err);
    if (!f || !u) return set_err(P, VP_EINVAL, "f and u must not be NULL");
    if (overlaps(f, 8 * (size_t)P->nbatch * P->nd, u, 8 * (size_t)P->nbatch * P->m))
        return set_err(P, VP_EINVAL, "f and u overlap");
    const size_t need = vp::carve_workspace(P, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (need > VP_NOALLOC_MAX_BYTES)
        return set_err(P, VP_EINVAL, "the evaluation workspace of this plan (" + std::to_string(need) +
                                         " bytes) exceeds the static workspace of vp_eval_noalloc (" +
                                         std::to_string((size_t)VP_NOALLOC_MAX_BYTES) + " bytes)");
    if (!P->scratch_dev) return set_err(P, VP_EINTERNAL, "static workspace address not resolved");
    // the same evaluation as vp_eval with the plan's workspace pointers
    // swapped for parts of the static array (restored afterwards; the kernels
    // have taken their arguments at launch)
    double *q0 = P->q, *acc0 = P->acc, *far0 = P->acc_far, *qi0 = P->qi;
    void *M0 = P->Mexp, *L0 = P->Lexp;
    vp::carve_workspace(P, static_cast<unsigned char *>(P->scratch_dev), &P->q, &P->acc, &P->acc_far, &P->Mexp,
                        &P->Lexp, &P->qi);
    vp_status st = guarded(P, [&] {
        // the expansions' padding rows must be zero (the plan zeroes its own
        // arrays once; the static array holds whatever the last call left)
        const int64_t ecount = (int64_t)P->tree.nbox * P->nbatch * P->PD;
        const int64_t mcount = P->mexp_boxes() * P->nbatch * P->PD;
        if (P->fp32) {
            vp::fill_f32(static_cast<float *>(P->Mexp), 0.f, mcount, P->stream);
            vp::fill_f32(static_cast<float *>(P->Lexp), 0.f, ecount, P->stream);
        } else {
            vp::fill_f64(static_cast<double *>(P->Mexp), 0.0, mcount, P->stream);
            vp::fill_f64(static_cast<double *>(P->Lexp), 0.0, ecount, P->stream);
        }
        if (P->qi) vp::fill_f64(P->qi + P->qi_zero * P->nbatch, 0.0, (int64_t)vp::QI_ZERO_PTS * P->nbatch, P->stream);
        P->timing_eval_begin();
        vp::prepare_charges(P, f, false);
        vp::run_fmm(P, false, false, f, u);
    });
    P->q = q0;
    P->acc = acc0;
    P->acc_far = far0;
    P->qi = qi0;
    P->Mexp = M0;
    P->Lexp = L0;
    return st;
}

extern "C" vp_status vp_eval_adjoint(vp_plan_t P, const double *g, double *df) {
    if (!P) return set_err(nullptr, VP_EINVAL, "plan is NULL");
    if (P->poisoned) return set_err(P, VP_EDEVICE, "plan is poisoned by an earlier device error: " + P->err);
    if (!g || !df) return set_err(P, VP_EINVAL, "g and df must not be NULL");
    if (overlaps(g, 8 * (size_t)P->nbatch * P->m, df, 8 * (size_t)P->nbatch * P->nd))
        return set_err(P, VP_EINVAL, "g and df overlap");
    return guarded(P, [&] {
        P->timing_eval_begin();
        vp::prepare_charges(P, g, true);
        vp::run_fmm(P, true, false, g, df);
    });
}

extern "C" vp_status vp_eval_grad_targets(vp_plan_t P, const double *f, double *grad) {
    if (!P) return set_err(nullptr, VP_EINVAL, "plan is NULL");
    if (P->yk.active)
        return set_err(P, VP_EUNSUPPORTED, "target gradients of the modified Helmholtz kernel are not built");
    if (P->poisoned) return set_err(P, VP_EDEVICE, "plan is poisoned by an earlier device error: " + P->err);
    if (!f || !grad) return set_err(P, VP_EINVAL, "f and grad must not be NULL");
    if (overlaps(f, 8 * (size_t)P->nbatch * P->nd, grad, 16 * (size_t)P->nbatch * P->m))
        return set_err(P, VP_EINVAL, "f and grad overlap");
    return guarded(P, [&] {
        P->timing_eval_begin();
        vp::prepare_charges(P, f, false, true);
        vp::run_fmm(P, false, true);
        vp::finish_grad(P, grad);
    });
}

extern "C" vp_status vp_correction_blocks(int32_t shape, int32_t p, const double *ref_x, const double *ref_y,
                                          const double *wref, int64_t ncell, const double *maps, double *out,
                                          void *stream) {
    return guarded(nullptr, [&] {
        vp::correction_blocks(shape, p, ref_x, ref_y, wref, ncell, maps, out, static_cast<hipStream_t>(stream));
    });
}

extern "C" vp_status vp_set_stream(vp_plan_t P, void *stream) {
    if (!P) return set_err(nullptr, VP_EINVAL, "plan is NULL");
    P->stream = static_cast<hipStream_t>(stream);
    P->opt.stream = stream;
    return VP_OK;
}

extern "C" vp_status vp_set_timing(vp_plan_t P, int32_t enable) {
    if (!P) return set_err(nullptr, VP_EINVAL, "plan is NULL");
    return guarded(P, [&] {
        VP_HIP(P->stream ? hipStreamSynchronize(P->stream) : hipDeviceSynchronize());
        release_timing(P);
        P->tcount = P->tdone = 0;
        P->tcur = -1;
        for (double &v : P->tms) v = 0.0;
        if (enable) {
            P->tev.assign((size_t)vp_plan_s::TRING * VP_NSTAGES * 2, nullptr);
            for (auto &e : P->tev) VP_HIP(hipEventCreate(&e));
            P->tslot_used.assign(vp_plan_s::TRING, 0);
            P->timing = true;
        }
    });
}

extern "C" vp_status vp_get_timing(vp_plan_t P, double *ms, int64_t *nevals) {
    if (!P || !ms || !nevals) return set_err(P, VP_EINVAL, "plan, ms and nevals must not be NULL");
    return guarded(P, [&] {
        if (P->timing) P->timing_collect(P->tcount);
        for (int st = 0; st < VP_NSTAGES; ++st) ms[st] = P->tms[st];
        *nevals = P->tdone;
    });
}

extern "C" vp_status vp_destroy(vp_plan_t P) {
    if (!P) return VP_OK;
    free_plan(P);
    return VP_OK;
}

extern "C" const char *vp_last_error(vp_plan_t P) {
    if (P) return P->err.c_str();
    return g_last_error.c_str();
}

extern "C" vp_status vp_get_info(vp_plan_t P, vp_plan_info_t *info) {
    if (!P || !info) return set_err(P, VP_EINVAL, "plan and info must not be NULL");
    std::memset(info, 0, sizeof(*info));
    info->n = P->n;
    info->m = P->m;
    info->nnz = P->nnz;
    info->nbatch = P->nbatch;
    info->order = P->p;
    info->precision = P->opt.precision;
    info->m2l_mode = P->m2l_mode;
    info->p2p_mode_used = P->near.active ? VP_P2P_TABLES : VP_P2P_PAIRWISE;
    info->max_leaf = P->opt.max_leaf;
    info->nbox = P->tree.nbox;
    info->nleaf = P->tree.nleaf;
    info->nlevels = P->tree.nlevels;
    info->self_targets = P->self ? 1 : 0;
    for (int k = 0; k < 4; ++k) info->list_len[k] = P->tree.llen[k];
    info->table_leaves = P->near.nleaf_tab;
    info->near_pairs = P->near_pairs;
    info->workspace_bytes = (int64_t)P->mem.bytes;
    info->m2l_translations = P->m2l_translations;
    info->m2l_tile_ops = P->m2l_tile_ops;
    info->m2l_coarse_translations = P->m2l[1].translations;
    info->m2l_coarse_tile_ops = P->m2l[1].tile_ops;
    info->split_level = P->split_level;
    info->corr_cells = P->ncell;
    info->corr_shared_cells = P->ncell_shared;
    info->corr_groups = P->nbatch == 1 ? P->ngrp : 0;
    info->corr_one_block = P->corr_op != nullptr ? 1 : 0;
    info->corr_folded = P->near.corr_folded ? 1 : 0;
    info->table_pattern = P->near.active ? P->near.npat : 0;
    info->corr_values_read = P->ncell > 0 ? P->corr_values_read : P->nnz;
    info->table_tile_ops = P->near.table_tile_ops;
    for (int k = 0; k < 3; ++k) info->root[k] = P->opt.root[k];
    info->table_pairs = P->table_pairs;
    info->n_in = P->nd;
    info->os_p = P->os_p;
    info->os_q = P->os_q;
    info->kernel = P->opt.kernel;
    info->lambda = P->opt.lambda;
    info->tuned = P->tuned;
    info->m2l_waves = P->m2l_nw;
    info->table_waves = P->table_nw;
    info->one_stream = P->one_stream ? 1 : 0;
    info->tune_ms = P->tune_ms;
    info->l2p_from_parents = P->near.par_l2p ? 1 : 0;
    if (P->yk.active) {
        info->m2l_translations = P->yk.m2l_translations;
        info->m2l_tile_ops = P->yk.m2l_tile_ops;
        info->m2l_coarse_translations = info->m2l_coarse_tile_ops = 0;
    }
    info->noalloc_bytes = (int64_t)vp::carve_workspace(P, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
    return VP_OK;
}

template <class T>
static void d2h(void *out, const T *d, int64_t count) {
    if (count > 0) VP_HIP(hipMemcpy(out, d, sizeof(T) * count, hipMemcpyDeviceToHost));
}

extern "C" vp_status vp_get_array(vp_plan_t P, int32_t which, void *out, int64_t *count) {
    if (!P || !count) return set_err(P, VP_EINVAL, "plan and count must not be NULL");
    if (P->poisoned) return set_err(P, VP_EDEVICE, "plan is poisoned: " + P->err);
    vp::Tree &T = P->tree;
    return guarded(P, [&] {
        VP_HIP(P->stream ? hipStreamSynchronize(P->stream) : hipDeviceSynchronize());
        int64_t c = 0;
        switch (which) {
            case VP_ARR_SRC_PERM: c = P->n; if (out) d2h(out, P->sperm, c); break;
            case VP_ARR_TGT_PERM: c = P->m; if (out) d2h(out, P->tperm, c); break;
            case VP_ARR_SRC_KEYS: c = P->n; if (out) d2h(out, P->skeys, c); break;
            case VP_ARR_TGT_KEYS: c = P->m; if (out) d2h(out, P->tkeys, c); break;
            case VP_ARR_LEVEL_BEGIN:
                c = T.nlevels + 1;
                if (out) std::memcpy(out, T.level_begin.data(), 4 * c);
                break;
            case VP_ARR_BOX: {
                c = (int64_t)T.nbox * 10;
                if (out) {
                    const int32_t *cols[10] = {T.level, T.ix, T.iy, T.parent, T.child, T.nchild, T.sb, T.se, T.tb, T.te};
                    std::vector<int32_t> tmp(T.nbox);
                    int32_t *o = static_cast<int32_t *>(out);
                    for (int k = 0; k < 10; ++k) {
                        d2h(tmp.data(), cols[k], T.nbox);
                        for (int b = 0; b < T.nbox; ++b) o[(int64_t)b * 10 + k] = tmp[b];
                    }
                }
                break;
            }
            case VP_ARR_U_PTR: case VP_ARR_V_PTR: case VP_ARR_W_PTR: case VP_ARR_X_PTR: {
                int k = (which - VP_ARR_U_PTR) / 2;
                c = T.nbox + 1;
                if (out) d2h(out, T.lptr[k], c);
                break;
            }
            case VP_ARR_U_IDX: case VP_ARR_V_IDX: case VP_ARR_W_IDX: case VP_ARR_X_IDX: {
                int k = (which - VP_ARR_U_IDX) / 2;
                c = T.llen[k];
                if (out) d2h(out, T.lidx[k], c);
                break;
            }
            case VP_ARR_MULTIPOLE:
            case VP_ARR_LOCAL: {
                c = (int64_t)T.nbox * P->nbatch * 2 * P->P;
                if (out) {
                    const size_t cnt = (size_t)T.nbox * P->nbatch * P->PD;
                    std::vector<double> h(cnt);
                    const void *src = which == VP_ARR_MULTIPOLE ? P->Mexp : P->Lexp;
                    if (P->fp32) {
                        std::vector<float> hf(cnt);
                        d2h(hf.data(), static_cast<const float *>(src), (int64_t)cnt);
                        for (size_t i = 0; i < cnt; ++i) h[i] = hf[i];
                    } else {
                        d2h(h.data(), static_cast<const double *>(src), (int64_t)cnt);
                    }
                    double *o = static_cast<double *>(out);
                    for (size_t col = 0; col < (size_t)T.nbox * P->nbatch; ++col)
                        for (int r = 0; r < 2 * P->P; ++r) o[col * 2 * P->P + r] = h[col * P->PD + r];
                }
                break;
            }
            default:
                throw Error(VP_EINVAL, "unknown array id");
        }
        *count = c;
    });
}

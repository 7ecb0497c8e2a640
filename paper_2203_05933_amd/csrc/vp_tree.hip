// Plan-time tree construction on the GPU: Morton keys, a stable LSD radix
// sort, level-by-level quadtree build and the U/V/W/X interaction lists of
// the adaptive FMM.  The paper evaluates its smooth rule (Section 3.2, eq.
// Tk_smooth_quad) with a point FMM over a static geometry (Section 1, static
// geometries; Section 5, set-up excluded from the timings); the tree is that
// FMM's set-up and is built once per plan.
//
// Tree definition (integer work, reproduced exactly):
//   q = clamp(floor(((v - v0) / side) * 2^30), 0, 2^30 - 1) in float64;
//   key = bit-interleave (x bit b -> key bit 2b, y bit b -> 2b+1);
//   points sorted by key, ties by input index;
//   a box splits while it holds more than max_leaf sources or targets (and
//   is above max_level); children are the non-empty quadrants in key order;
//   boxes are numbered level by level, Morton order inside a level.
// Lists (adjacent = closed squares intersect):
//   U(b), leaf b: leaves adjacent to b (b included);
//   V(b): boxes on b's level not adjacent to b whose parents are adjacent;
//   W(b), leaf b: finer boxes not adjacent to b whose parent is adjacent to b;
//   X(b): coarser leaves not adjacent to b that are adjacent to b's parent.

#include "vp_internal.hpp"

#include <algorithm>

namespace vp {

// ----------------------------------------------------------------------------
// small utilities
// ----------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = v;
}
__global__ void k_fill_f64(double *p, double v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = v;
}
__global__ void k_fill_f32(float *p, float v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = v;
}

static unsigned grid_for(int64_t n, int bs = 256) {
    int64_t g = (n + bs - 1) / bs;
    if (g < 1) g = 1;
    if (g > 65535 * 16) g = 65535 * 16;
    return (unsigned)g;
}

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
    VP_LAUNCH_CHECK();
}
void fill_f64(double *p, double v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
    VP_LAUNCH_CHECK();
}
void fill_f32(float *p, float v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
    VP_LAUNCH_CHECK();
}

// ----------------------------------------------------------------------------
// Exclusive scan of int32 (three phases: tile scan, scan of tile sums, add).
// out must hold n+1 entries; out[n] receives the total.
// ----------------------------------------------------------------------------
constexpr int SCAN_BS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BS * SCAN_ITEMS;

__global__ void k_scan_tiles(const int32_t *in, int32_t *out, int32_t *tile_sum, int n) {
    __shared__ int32_t s[SCAN_BS];
    int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t tot = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int i = base + k;
        v[k] = (i < n) ? in[i] : 0;
        tot += v[k];
    }
    s[threadIdx.x] = tot;
    __syncthreads();
    // Hillis-Steele inclusive scan of the thread totals
    for (int off = 1; off < SCAN_BS; off <<= 1) {
        int32_t t = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    int32_t run = s[threadIdx.x] - tot;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        int i = base + k;
        if (i < n) out[i] = run;
        run += v[k];
    }
    if (threadIdx.x == SCAN_BS - 1) tile_sum[blockIdx.x] = s[SCAN_BS - 1];
}

__global__ void k_scan_add(int32_t *out, const int32_t *tile_off, int n) {
    int i = blockIdx.x * SCAN_TILE + threadIdx.x;
    int32_t add = tile_off[blockIdx.x];
    for (int k = 0; k < SCAN_ITEMS; ++k, i += SCAN_BS)
        if (i < n) out[i] += add;
}

__global__ void k_set_total(int32_t *out, const int32_t *in, int n) {
    // out[n] = out[n-1] + in[n-1]
    if (n > 0) out[n] = out[n - 1] + in[n - 1];
    else out[0] = 0;
}

void exclusive_scan_i32(const int32_t *in, int32_t *out, int n, hipStream_t s) {
    if (n <= 0) {
        fill_i32(out, 0, 1, s);
        return;
    }
    int ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    TempArena tmp;
    int32_t *ts = tmp.alloc<int32_t>(ntiles + 1);
    int32_t *to = tmp.alloc<int32_t>(ntiles + 1);
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(SCAN_BS), 0, s, in, out, ts, n);
    VP_LAUNCH_CHECK();
    if (ntiles > 1) {
        exclusive_scan_i32(ts, to, ntiles, s);
        hipLaunchKernelGGL(k_scan_add, dim3(ntiles), dim3(SCAN_BS), 0, s, out, to, n);
        VP_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_set_total, dim3(1), dim3(1), 0, s, out, in, n);
    VP_LAUNCH_CHECK();
    VP_HIP(hipStreamSynchronize(s));  // temporaries are freed on return
}

// ----------------------------------------------------------------------------
// Stable LSD radix sort of (uint64 key, int32 value), 8-bit digits.
// Stability inside a tile comes from wave ballots (lanes with equal digits
// are ranked by lane order) and a running per-digit count across rounds.
// ----------------------------------------------------------------------------
constexpr int RS_BS = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_BS * RS_ITEMS;
constexpr int RS_WAVES = RS_BS / 64;

__global__ void k_rs_hist(const uint64_t *keys, int n, int shift, int32_t *hist, int nblocks) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
        int i = base + r * RS_BS + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_rs_scatter(const uint64_t *kin, const int32_t *vin, uint64_t *kout,
                             int32_t *vout, int n, int shift, const int32_t *offs, int nblocks) {
    __shared__ int32_t run[256];
    __shared__ int32_t wcnt[RS_WAVES][256];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    run[threadIdx.x] = offs[threadIdx.x * nblocks + blockIdx.x];
    const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int base = blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ITEMS; ++r) {
        for (int w = 0; w < RS_WAVES; ++w) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        int i = base + r * RS_BS + threadIdx.x;
        bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0;
        int32_t val = valid ? vin[i] : 0;
        unsigned d = (unsigned)((key >> shift) & 255u);
        uint64_t peers = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            bool b = (d >> bit) & 1u;
            uint64_t bal = __ballot(b);
            peers &= b ? bal : ~bal;
        }
        int rank = __popcll(peers & lt_mask);
        bool leader = valid && ((peers & lt_mask) == 0);
        if (leader) wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pos = run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        int add = 0;
        for (int w = 0; w < RS_WAVES; ++w) add += wcnt[w][threadIdx.x];
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

void radix_sort_pairs_u64(uint64_t *keys, int32_t *vals, int n, int nbits, hipStream_t s) {
    if (n <= 1) return;
    TempArena tmp;
    uint64_t *k2 = tmp.alloc<uint64_t>(n);
    int32_t *v2 = tmp.alloc<int32_t>(n);
    int nblocks = (n + RS_TILE - 1) / RS_TILE;
    int32_t *hist = tmp.alloc<int32_t>((size_t)256 * nblocks);
    int32_t *offs = tmp.alloc<int32_t>((size_t)256 * nblocks + 1);
    uint64_t *ka = keys, *kb = k2;
    int32_t *va = vals, *vb = v2;
    int passes = (nbits + 7) / 8;
    for (int ps = 0; ps < passes; ++ps) {
        int shift = 8 * ps;
        hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(RS_BS), 0, s, ka, n, shift, hist, nblocks);
        VP_LAUNCH_CHECK();
        exclusive_scan_i32(hist, offs, 256 * nblocks, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(RS_BS), 0, s, ka, va, kb, vb, n, shift,
                           offs, nblocks);
        VP_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        VP_HIP(hipMemcpyAsync(keys, ka, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
        VP_HIP(hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    }
    VP_HIP(hipStreamSynchronize(s));
}

// ----------------------------------------------------------------------------
// Morton keys
// ----------------------------------------------------------------------------
__host__ __device__ inline uint64_t spread_bits(uint64_t v) {
    // insert a zero bit above each of the low 32 bits
    v &= 0xFFFFFFFFull;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}
__host__ __device__ inline uint64_t interleave(uint32_t ix, uint32_t iy) {
    return spread_bits(ix) | (spread_bits(iy) << 1);
}

__device__ inline uint32_t quantise(double v, double v0, double side) {
    double t = (v - v0) / side;
    t = t * 1073741824.0;  // 2^30, exact
    double q = floor(t);
    if (!(q >= 0.0)) q = 0.0;
    if (q > 1073741823.0) q = 1073741823.0;
    return (uint32_t)q;
}

__global__ void k_keys(const double *x, const double *y, int n, double x0, double y0, double side,
                       uint64_t *keys, int32_t *idx) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = interleave(quantise(x[i], x0, side), quantise(y[i], y0, side));
    idx[i] = i;
}

__global__ void k_gather_f64(const double *in, const int32_t *perm, double *out, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[perm[i]];
}
__global__ void k_invert_perm(const int32_t *perm, int32_t *inv, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) inv[perm[i]] = i;
}

// ----------------------------------------------------------------------------
// Level-by-level tree build
// ----------------------------------------------------------------------------
__device__ inline int lower_bound_u64(const uint64_t *a, int lo, int hi, uint64_t v) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

struct LevelArrays {
    int32_t *ix, *iy, *parent, *sb, *se, *tb, *te;
};

// For each box of the level: decide the split, compute the four quadrant
// ranges and count the non-empty ones.
__global__ void k_split_count(LevelArrays L, int nb, int level, int max_leaf, int max_level,
                              const uint64_t *skeys, const uint64_t *tkeys, int32_t *qr /*[nb][4][4]*/,
                              int32_t *cnt) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    int s0 = L.sb[k], s1 = L.se[k], t0 = L.tb[k], t1 = L.te[k];
    bool split = ((s1 - s0) > max_leaf || (t1 - t0) > max_leaf) && level < max_level;
    int c = 0;
    if (split) {
        uint64_t prefix = interleave((uint32_t)L.ix[k], (uint32_t)L.iy[k]) << 2;
        int shift = 2 * (LBITS - level - 1);
        int ps = s0, pt = t0;
        for (int q = 0; q < 4; ++q) {
            uint64_t hi = ((prefix | (uint64_t)q) + 1ull) << shift;
            int cs1 = lower_bound_u64(skeys, ps, s1, hi);
            int ct1 = lower_bound_u64(tkeys, pt, t1, hi);
            qr[(k * 4 + q) * 4 + 0] = ps;
            qr[(k * 4 + q) * 4 + 1] = cs1;
            qr[(k * 4 + q) * 4 + 2] = pt;
            qr[(k * 4 + q) * 4 + 3] = ct1;
            if ((cs1 - ps) + (ct1 - pt) > 0) ++c;
            ps = cs1;
            pt = ct1;
        }
    }
    cnt[k] = c;
}

__global__ void k_split_write(LevelArrays L, int nb, int level_base, const int32_t *qr,
                              const int32_t *cnt, const int32_t *off, LevelArrays C,
                              int32_t *child_local) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    if (cnt[k] == 0) {
        child_local[k] = -1;
        return;
    }
    int j = off[k];
    child_local[k] = j;
    for (int q = 0; q < 4; ++q) {
        const int32_t *r = qr + (k * 4 + q) * 4;
        if ((r[1] - r[0]) + (r[3] - r[2]) == 0) continue;
        C.ix[j] = 2 * L.ix[k] + (q & 1);
        C.iy[j] = 2 * L.iy[k] + (q >> 1);
        C.parent[j] = level_base + k;
        C.sb[j] = r[0];
        C.se[j] = r[1];
        C.tb[j] = r[2];
        C.te[j] = r[3];
        ++j;
    }
}

__global__ void k_box_finish(int nbox, const int32_t *level_of, const int32_t *ix, const int32_t *iy,
                             double x0, double y0, const double *side, uint64_t *key, double *cx,
                             double *cy) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    int l = level_of[b];
    double h = side[l];
    key[b] = interleave((uint32_t)ix[b], (uint32_t)iy[b]);
    cx[b] = x0 + ((double)ix[b] + 0.5) * h;
    cy[b] = y0 + ((double)iy[b] + 0.5) * h;
}

// ----------------------------------------------------------------------------
// Interaction lists
// ----------------------------------------------------------------------------
struct TreeView {
    const int32_t *level_begin;
    int nlevels;
    const int32_t *level, *ix, *iy, *parent, *child, *nchild;
    const uint64_t *key;
};

__device__ inline int find_box(const TreeView &T, int l, int ix, int iy) {
    if (l >= T.nlevels) return -1;
    int n = 1 << l;
    if (ix < 0 || iy < 0 || ix >= n || iy >= n) return -1;
    uint64_t k = interleave((uint32_t)ix, (uint32_t)iy);
    int lo = T.level_begin[l], hi = T.level_begin[l + 1];
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (T.key[mid] < k) lo = mid + 1;
        else hi = mid;
    }
    if (lo < T.level_begin[l + 1] && T.key[lo] == k) return lo;
    return -1;
}

__device__ inline bool adjacent_boxes(const TreeView &T, int a, int b) {
    int la = T.level[a], lb = T.level[b];
    int L = la > lb ? la : lb;
    int sa = L - la, sb = L - lb;
    int64_t ax0 = (int64_t)T.ix[a] << sa, ax1 = (int64_t)(T.ix[a] + 1) << sa;
    int64_t ay0 = (int64_t)T.iy[a] << sa, ay1 = (int64_t)(T.iy[a] + 1) << sa;
    int64_t bx0 = (int64_t)T.ix[b] << sb, bx1 = (int64_t)(T.ix[b] + 1) << sb;
    int64_t by0 = (int64_t)T.iy[b] << sb, by1 = (int64_t)(T.iy[b] + 1) << sb;
    return ax0 <= bx1 && bx0 <= ax1 && ay0 <= by1 && by0 <= ay1;
}

// Sink for list entries: counting pass or writing pass.
struct ListSink {
    int32_t *idx[4];   // nullptr in the counting pass
    int32_t pos[4];
    int32_t cnt[4];
    int32_t cap[4];    // entries reserved by the counting pass (writing pass)
    int32_t *voff;
    int32_t *vslot;    // [NOFF] row of the slot table for this box (writing pass)
    __device__ void add(int list, int a, int code = -1) {
        if (idx[list] && cnt[list] < cap[list]) {
            idx[list][pos[list] + cnt[list]] = a;
            if (list == 1) {
                voff[pos[1] + cnt[1]] = code;
                if (code >= 0 && code < NOFF) vslot[code] = a;
            }
        }
        cnt[list]++;
    }
};

constexpr int LIST_STACK = 128;

// Leaves adjacent to box b at coarser levels, found by walking up from b's
// eight neighbour cells that hold no box on b's level.  Returns count.
__device__ int coarse_adjacent_leaves(const TreeView &T, int b, int *out, int cap) {
    int l = T.level[b];
    int nout = 0;
    for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
            if (dx == 0 && dy == 0) continue;
            int cx = T.ix[b] + dx, cy = T.iy[b] + dy;
            int n = 1 << l;
            if (cx < 0 || cy < 0 || cx >= n || cy >= n) continue;
            if (find_box(T, l, cx, cy) >= 0) continue;
            for (int lu = l - 1; lu >= 0; --lu) {
                int a = find_box(T, lu, cx >> (l - lu), cy >> (l - lu));
                if (a < 0) continue;
                if (T.nchild[a] == 0) {
                    bool dup = false;
                    for (int k = 0; k < nout; ++k) dup |= (out[k] == a);
                    if (!dup && nout < cap) out[nout++] = a;
                }
                break;
            }
        }
    return nout;
}

__device__ void enumerate_lists(const TreeView &T, int b, ListSink &S, int32_t *err) {
    int l = T.level[b];
    bool leaf = T.nchild[b] == 0;
    int bix = T.ix[b], biy = T.iy[b];
    if (leaf) {
        // same-level colleagues
        int stack[LIST_STACK];
        int sp = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int c = find_box(T, l, bix + dx, biy + dy);
                if (c < 0) continue;
                if (T.nchild[c] == 0) S.add(0, c);
                else if (sp < LIST_STACK) stack[sp++] = c;
                else atomicOr(err, 1);
            }
        // descend non-leaf colleagues: adjacent leaves -> U, separated -> W
        while (sp > 0) {
            int c = stack[--sp];
            int c0 = T.child[c], nc = T.nchild[c];
            for (int d = c0; d < c0 + nc; ++d) {
                if (adjacent_boxes(T, d, b)) {
                    if (T.nchild[d] == 0) S.add(0, d);
                    else if (sp < LIST_STACK) stack[sp++] = d;
                    else atomicOr(err, 1);
                } else {
                    S.add(2, d);
                }
            }
        }
        // coarser adjacent leaves
        int coarse[8];
        int nco = coarse_adjacent_leaves(T, b, coarse, 8);
        for (int k = 0; k < nco; ++k) S.add(0, coarse[k]);
    }
    int P = T.parent[b];
    if (P >= 0) {
        int lp = l - 1;
        int pix = T.ix[P], piy = T.iy[P];
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                int C = find_box(T, lp, pix + dx, piy + dy);
                if (C < 0) continue;
                if (T.nchild[C] == 0) {
                    // colleague of the parent that is a leaf: X candidate
                    if (!adjacent_boxes(T, C, b)) S.add(3, C);
                    continue;
                }
                int c0 = T.child[C], nc = T.nchild[C];
                for (int d = c0; d < c0 + nc; ++d) {
                    int ox = T.ix[d] - bix, oy = T.iy[d] - biy;
                    bool adj = ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1;
                    if (!adj) S.add(1, d, offset_code(ox, oy));
                }
            }
        int coarse[8];
        int nco = coarse_adjacent_leaves(T, P, coarse, 8);
        for (int k = 0; k < nco; ++k)
            if (!adjacent_boxes(T, coarse[k], b)) S.add(3, coarse[k]);
    }
}

__global__ void k_lists_count(TreeView T, int nbox, int32_t *cnt /*[4][nbox]*/, int32_t *err) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    ListSink S;
    for (int k = 0; k < 4; ++k) {
        S.idx[k] = nullptr;
        S.pos[k] = 0;
        S.cnt[k] = 0;
        S.cap[k] = 0;
    }
    S.voff = nullptr;
    S.vslot = nullptr;
    enumerate_lists(T, b, S, err);
    for (int k = 0; k < 4; ++k) cnt[k * nbox + b] = S.cnt[k];
}

__device__ void sort_segment(int32_t *a, int32_t *aux, int n) {
    for (int i = 1; i < n; ++i) {
        int32_t v = a[i];
        int32_t w = aux ? aux[i] : 0;
        int j = i - 1;
        while (j >= 0 && a[j] > v) {
            a[j + 1] = a[j];
            if (aux) aux[j + 1] = aux[j];
            --j;
        }
        a[j + 1] = v;
        if (aux) aux[j + 1] = w;
    }
}

__global__ void k_lists_fill(TreeView T, int nbox, int32_t *const *ptr, int32_t *const *idx,
                             int32_t *voff, int32_t *vslot, int32_t *err) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    ListSink S;
    for (int k = 0; k < 4; ++k) {
        S.idx[k] = idx[k];
        S.pos[k] = ptr[k][b];
        S.cnt[k] = 0;
        S.cap[k] = ptr[k][b + 1] - ptr[k][b];
    }
    S.voff = voff;
    S.vslot = vslot + (int64_t)b * NOFF;
    enumerate_lists(T, b, S, err);
    for (int k = 0; k < 4; ++k) {
        int n = ptr[k][b + 1] - ptr[k][b];
        if (n != S.cnt[k]) atomicOr(err, 2);
        sort_segment(idx[k] + ptr[k][b], k == 1 ? voff + ptr[1][b] : nullptr, n);
    }
}

// ----------------------------------------------------------------------------
// Host driver
// ----------------------------------------------------------------------------
static void bounding_square(const double *x, const double *y, int64_t n, const double *tx,
                            const double *ty, int64_t m, double root[3]) {
    double lo_x = x[0], hi_x = x[0], lo_y = y[0], hi_y = y[0];
    for (int64_t i = 0; i < n; ++i) {
        lo_x = std::min(lo_x, x[i]);
        hi_x = std::max(hi_x, x[i]);
        lo_y = std::min(lo_y, y[i]);
        hi_y = std::max(hi_y, y[i]);
    }
    if (tx)
        for (int64_t i = 0; i < m; ++i) {
            lo_x = std::min(lo_x, tx[i]);
            hi_x = std::max(hi_x, tx[i]);
            lo_y = std::min(lo_y, ty[i]);
            hi_y = std::max(hi_y, ty[i]);
        }
    double side = std::max(hi_x - lo_x, hi_y - lo_y);
    if (side <= 0) side = 1.0;
    side *= 1.0 + 1e-9;
    double cx = 0.5 * (lo_x + hi_x), cy = 0.5 * (lo_y + hi_y);
    root[0] = cx - 0.5 * side;
    root[1] = cy - 0.5 * side;
    root[2] = side;
}

void build_tree(vp_plan_s *P, const double *hx, const double *hy, const double *htx,
                const double *hty) {
    hipStream_t s = P->stream;
    const int n = (int)P->n, m = (int)P->m;
    if (!(P->opt.root[2] > 0)) bounding_square(hx, hy, n, htx, hty, m, P->opt.root);
    const double x0 = P->opt.root[0], y0 = P->opt.root[1], side = P->opt.root[2];
    const int max_level = P->opt.max_level > 0 ? P->opt.max_level : LBITS;
    const int max_leaf = P->opt.max_leaf;

    TempArena tmp;
    // --- points, keys, sort
    double *ux = tmp.alloc<double>(n), *uy = tmp.alloc<double>(n), *uw = P->w_user;
    VP_HIP(hipMemcpyAsync(ux, hx, sizeof(double) * n, hipMemcpyHostToDevice, s));
    VP_HIP(hipMemcpyAsync(uy, hy, sizeof(double) * n, hipMemcpyHostToDevice, s));
    P->skeys = P->mem.alloc<uint64_t>(n);
    P->sperm = P->mem.alloc<int32_t>(n);
    P->sinv = P->mem.alloc<int32_t>(n);
    hipLaunchKernelGGL(k_keys, dim3(grid_for(n)), dim3(256), 0, s, ux, uy, n, x0, y0, side, P->skeys,
                       P->sperm);
    VP_LAUNCH_CHECK();
    radix_sort_pairs_u64(P->skeys, P->sperm, n, 2 * LBITS, s);
    P->sx = P->mem.alloc<double>(n);
    P->sy = P->mem.alloc<double>(n);
    P->sw = P->mem.alloc<double>(n);
    hipLaunchKernelGGL(k_gather_f64, dim3(grid_for(n)), dim3(256), 0, s, ux, P->sperm, P->sx, n);
    hipLaunchKernelGGL(k_gather_f64, dim3(grid_for(n)), dim3(256), 0, s, uy, P->sperm, P->sy, n);
    hipLaunchKernelGGL(k_gather_f64, dim3(grid_for(n)), dim3(256), 0, s, uw, P->sperm, P->sw, n);
    hipLaunchKernelGGL(k_invert_perm, dim3(grid_for(n)), dim3(256), 0, s, P->sperm, P->sinv, n);
    VP_LAUNCH_CHECK();
    if (P->self) {
        P->tx = P->sx;
        P->ty = P->sy;
        P->tperm = P->sperm;
        P->tinv = P->sinv;
        P->tkeys = P->skeys;
    } else {
        double *vx = tmp.alloc<double>(m), *vy = tmp.alloc<double>(m);
        VP_HIP(hipMemcpyAsync(vx, htx, sizeof(double) * m, hipMemcpyHostToDevice, s));
        VP_HIP(hipMemcpyAsync(vy, hty, sizeof(double) * m, hipMemcpyHostToDevice, s));
        P->tkeys = P->mem.alloc<uint64_t>(m);
        P->tperm = P->mem.alloc<int32_t>(m);
        P->tinv = P->mem.alloc<int32_t>(m);
        hipLaunchKernelGGL(k_keys, dim3(grid_for(m)), dim3(256), 0, s, vx, vy, m, x0, y0, side,
                           P->tkeys, P->tperm);
        VP_LAUNCH_CHECK();
        radix_sort_pairs_u64(P->tkeys, P->tperm, m, 2 * LBITS, s);
        P->tx = P->mem.alloc<double>(m);
        P->ty = P->mem.alloc<double>(m);
        hipLaunchKernelGGL(k_gather_f64, dim3(grid_for(m)), dim3(256), 0, s, vx, P->tperm, P->tx, m);
        hipLaunchKernelGGL(k_gather_f64, dim3(grid_for(m)), dim3(256), 0, s, vy, P->tperm, P->ty, m);
        hipLaunchKernelGGL(k_invert_perm, dim3(grid_for(m)), dim3(256), 0, s, P->tperm, P->tinv, m);
        VP_LAUNCH_CHECK();
    }

    // --- levels
    struct HostLevel {
        int nb;
        LevelArrays a;
        int32_t *child_local;
        int32_t *nchild;
    };
    std::vector<HostLevel> levels;
    {
        HostLevel L0;
        L0.nb = 1;
        L0.a.ix = tmp.alloc<int32_t>(1);
        L0.a.iy = tmp.alloc<int32_t>(1);
        L0.a.parent = tmp.alloc<int32_t>(1);
        L0.a.sb = tmp.alloc<int32_t>(1);
        L0.a.se = tmp.alloc<int32_t>(1);
        L0.a.tb = tmp.alloc<int32_t>(1);
        L0.a.te = tmp.alloc<int32_t>(1);
        int32_t h[7] = {0, 0, -1, 0, n, 0, m};
        VP_HIP(hipMemcpyAsync(L0.a.ix, &h[0], 4, hipMemcpyHostToDevice, s));
        VP_HIP(hipMemcpyAsync(L0.a.iy, &h[1], 4, hipMemcpyHostToDevice, s));
        VP_HIP(hipMemcpyAsync(L0.a.parent, &h[2], 4, hipMemcpyHostToDevice, s));
        VP_HIP(hipMemcpyAsync(L0.a.sb, &h[3], 4, hipMemcpyHostToDevice, s));
        VP_HIP(hipMemcpyAsync(L0.a.se, &h[4], 4, hipMemcpyHostToDevice, s));
        VP_HIP(hipMemcpyAsync(L0.a.tb, &h[5], 4, hipMemcpyHostToDevice, s));
        VP_HIP(hipMemcpyAsync(L0.a.te, &h[6], 4, hipMemcpyHostToDevice, s));
        VP_HIP(hipStreamSynchronize(s));
        levels.push_back(L0);
    }
    int base = 0;
    for (int lev = 0;; ++lev) {
        HostLevel &L = levels.back();
        int nb = L.nb;
        int32_t *qr = tmp.alloc<int32_t>((size_t)nb * 16);
        L.nchild = tmp.alloc<int32_t>(nb);
        int32_t *off = tmp.alloc<int32_t>(nb + 1);
        L.child_local = tmp.alloc<int32_t>(nb);
        hipLaunchKernelGGL(k_split_count, dim3(grid_for(nb)), dim3(256), 0, s, L.a, nb, lev, max_leaf,
                           max_level, P->skeys, P->tkeys, qr, L.nchild);
        VP_LAUNCH_CHECK();
        exclusive_scan_i32(L.nchild, off, nb, s);
        int32_t total = 0;
        VP_HIP(hipMemcpy(&total, off + nb, 4, hipMemcpyDeviceToHost));
        HostLevel C{};
        C.nb = total;
        if (total > 0) {
            C.a.ix = tmp.alloc<int32_t>(total);
            C.a.iy = tmp.alloc<int32_t>(total);
            C.a.parent = tmp.alloc<int32_t>(total);
            C.a.sb = tmp.alloc<int32_t>(total);
            C.a.se = tmp.alloc<int32_t>(total);
            C.a.tb = tmp.alloc<int32_t>(total);
            C.a.te = tmp.alloc<int32_t>(total);
        }
        hipLaunchKernelGGL(k_split_write, dim3(grid_for(nb)), dim3(256), 0, s, L.a, nb, base, qr,
                           L.nchild, off, C.a, L.child_local);
        VP_LAUNCH_CHECK();
        base += nb;
        if (total == 0) break;
        levels.push_back(C);
    }
    VP_HIP(hipStreamSynchronize(s));

    // --- concatenate levels
    Tree &T = P->tree;
    T.nlevels = (int)levels.size();
    T.level_begin.assign(T.nlevels + 1, 0);
    for (int l = 0; l < T.nlevels; ++l) T.level_begin[l + 1] = T.level_begin[l] + levels[l].nb;
    T.nbox = T.level_begin[T.nlevels];
    const int nbox = T.nbox;
    T.level = P->mem.alloc<int32_t>(nbox);
    T.ix = P->mem.alloc<int32_t>(nbox);
    T.iy = P->mem.alloc<int32_t>(nbox);
    T.parent = P->mem.alloc<int32_t>(nbox);
    T.child = P->mem.alloc<int32_t>(nbox);
    T.nchild = P->mem.alloc<int32_t>(nbox);
    T.sb = P->mem.alloc<int32_t>(nbox);
    T.se = P->mem.alloc<int32_t>(nbox);
    T.tb = P->mem.alloc<int32_t>(nbox);
    T.te = P->mem.alloc<int32_t>(nbox);
    T.key = P->mem.alloc<uint64_t>(nbox);
    T.cx = P->mem.alloc<double>(nbox);
    T.cy = P->mem.alloc<double>(nbox);
    T.d_level_begin = P->mem.alloc<int32_t>(T.nlevels + 1);
    VP_HIP(hipMemcpyAsync(T.d_level_begin, T.level_begin.data(), 4 * (T.nlevels + 1),
                          hipMemcpyHostToDevice, s));
    for (int l = 0; l < T.nlevels; ++l) {
        HostLevel &L = levels[l];
        int o = T.level_begin[l];
        size_t bytes = 4 * (size_t)L.nb;
        VP_HIP(hipMemcpyAsync(T.ix + o, L.a.ix, bytes, hipMemcpyDeviceToDevice, s));
        VP_HIP(hipMemcpyAsync(T.iy + o, L.a.iy, bytes, hipMemcpyDeviceToDevice, s));
        VP_HIP(hipMemcpyAsync(T.parent + o, L.a.parent, bytes, hipMemcpyDeviceToDevice, s));
        VP_HIP(hipMemcpyAsync(T.sb + o, L.a.sb, bytes, hipMemcpyDeviceToDevice, s));
        VP_HIP(hipMemcpyAsync(T.se + o, L.a.se, bytes, hipMemcpyDeviceToDevice, s));
        VP_HIP(hipMemcpyAsync(T.tb + o, L.a.tb, bytes, hipMemcpyDeviceToDevice, s));
        VP_HIP(hipMemcpyAsync(T.te + o, L.a.te, bytes, hipMemcpyDeviceToDevice, s));
        VP_HIP(hipMemcpyAsync(T.nchild + o, L.nchild, bytes, hipMemcpyDeviceToDevice, s));
        fill_i32(T.level + o, l, L.nb, s);
        // child indices: local offsets of the next level -> global
        std::vector<int32_t> hc(L.nb);
        VP_HIP(hipMemcpyAsync(hc.data(), L.child_local, bytes, hipMemcpyDeviceToHost, s));
        VP_HIP(hipStreamSynchronize(s));
        int nb_next = T.level_begin[std::min(l + 1, T.nlevels)];
        for (auto &c : hc)
            if (c >= 0) c += nb_next;
        VP_HIP(hipMemcpyAsync(T.child + o, hc.data(), bytes, hipMemcpyHostToDevice, s));
        VP_HIP(hipStreamSynchronize(s));
    }
    T.side.resize(T.nlevels);
    std::vector<double> logside(T.nlevels);
    for (int l = 0; l < T.nlevels; ++l) {
        T.side[l] = std::ldexp(side, -l);
        logside[l] = std::log(T.side[l]);
    }
    T.d_side = P->mem.alloc<double>(T.nlevels);
    T.d_logside = P->mem.alloc<double>(T.nlevels);
    VP_HIP(hipMemcpyAsync(T.d_side, T.side.data(), 8 * T.nlevels, hipMemcpyHostToDevice, s));
    VP_HIP(hipMemcpyAsync(T.d_logside, logside.data(), 8 * T.nlevels, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_box_finish, dim3(grid_for(nbox)), dim3(256), 0, s, nbox, T.level, T.ix, T.iy,
                       x0, y0, T.d_side, T.key, T.cx, T.cy);
    VP_LAUNCH_CHECK();

    // --- lists
    TreeView V{T.d_level_begin, T.nlevels, T.level, T.ix, T.iy, T.parent, T.child, T.nchild, T.key};
    int32_t *cnt = tmp.alloc<int32_t>((size_t)4 * nbox);
    fill_i32(P->err_flag, 0, 1, s);
    hipLaunchKernelGGL(k_lists_count, dim3(grid_for(nbox, 64)), dim3(64), 0, s, V, nbox, cnt,
                       P->err_flag);
    VP_LAUNCH_CHECK();
    for (int k = 0; k < 4; ++k) {
        T.lptr[k] = P->mem.alloc<int32_t>(nbox + 1);
        exclusive_scan_i32(cnt + (size_t)k * nbox, T.lptr[k], nbox, s);
        int32_t tot = 0;
        VP_HIP(hipMemcpy(&tot, T.lptr[k] + nbox, 4, hipMemcpyDeviceToHost));
        T.llen[k] = tot;
        T.lidx[k] = P->mem.alloc<int32_t>(tot);
    }
    T.v_off = P->mem.alloc<int32_t>(T.llen[1]);
    T.v_slot = P->mem.alloc<int32_t>((size_t)nbox * NOFF);
    fill_i32(T.v_slot, -1, (int64_t)nbox * NOFF, s);
    int32_t **dptr = tmp.alloc<int32_t *>(8);
    int32_t *hptrs[8] = {T.lptr[0], T.lptr[1], T.lptr[2], T.lptr[3],
                         T.lidx[0], T.lidx[1], T.lidx[2], T.lidx[3]};
    VP_HIP(hipMemcpyAsync(dptr, hptrs, sizeof(hptrs), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_lists_fill, dim3(grid_for(nbox, 64)), dim3(64), 0, s, V, nbox, dptr, dptr + 4,
                       T.v_off, T.v_slot, P->err_flag);
    VP_LAUNCH_CHECK();
    int32_t errv = 0;
    VP_HIP(hipMemcpyAsync(&errv, P->err_flag, 4, hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));
    if (errv) throw Error(VP_EINTERNAL, "interaction-list traversal exceeded its stack (tree too deep)");

    // leaves
    std::vector<int32_t> hn(nbox);
    VP_HIP(hipMemcpy(hn.data(), T.nchild, 4 * (size_t)nbox, hipMemcpyDeviceToHost));
    std::vector<int32_t> lv;
    for (int b = 0; b < nbox; ++b)
        if (hn[b] == 0) lv.push_back(b);
    T.nleaf = (int)lv.size();
    T.leaves = P->mem.alloc<int32_t>(T.nleaf);
    VP_HIP(hipMemcpy(T.leaves, lv.data(), 4 * lv.size(), hipMemcpyHostToDevice));
}

}  // namespace vp

// Plan-time set-up of the congruent-leaf path.
//
// The paper's box cells all carry one reference rule mapped by
// R^k(zeta) = o_k + h zeta (Section 4.2, eq. Rk_box), and it builds its box
// corrections once as a lookup table because G(r, r0) = G(r - r0) is
// translation invariant (Section 4.2, eq. Vkhat_box).  The same invariance
// makes the smooth-rule near field between two leaves that are congruent
// copies of one node pattern a FIXED matrix per (level, relative position):
//     u_i += sum_j K_o[i][j] q_j,  K_o[i][j] = -(1/(4 pi)) log(h^2 |c_o + m xi_j - xi_i|^2)
// (zero for a zero-distance pair), where xi are pattern coordinates in box
// units, h the target leaf's side, m the source/target size ratio (1, or 2
// and 1/2 for adjacent leaves one level apart) and c_o the source centre
// relative to the target's in units of h.  Likewise the scaled P2M and L2P
// of such a leaf are fixed matrices (powers of the pattern).  All three run
// on matrix cores through the gather-GEMM kernel.  Leaves that are not
// copies of the pattern, and pairs further apart in level, keep the
// pairwise / series kernels.
//
// A leaf matches the reference pattern when it holds exactly npat points
// whose box-relative coordinates (x - c)/h agree with the pattern's to
// within a few units in the last place of the node coordinates:
//     |(x - c)/h - xi| <= PATTERN_ULPS * 2^-52 * (R / h + 1),
// R the largest coordinate magnitude of the root square.  That is the
// rounding the node coordinates themselves carry (x = c + h xi rounded, for
// this leaf and for the reference leaf), so the matrices, which use the
// pattern coordinates, change a logarithm by no more than the rounding of the
// coordinate difference in the direct sum does.  A leaf whose nodes deviate
// by more keeps the pairwise kernel, which uses its own coordinates.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <vector>

#include "vp_internal.hpp"

namespace vp {

constexpr double PATTERN_ULPS = 8.0;

__global__ void k_match_pattern(const int32_t *__restrict__ leaves, int nleaf, const int32_t *__restrict__ b0,
                                const int32_t *__restrict__ b1, const double *__restrict__ px,
                                const double *__restrict__ py, const double *__restrict__ cx,
                                const double *__restrict__ cy, const int32_t *__restrict__ level,
                                const double *__restrict__ side, const double *__restrict__ rx,
                                const double *__restrict__ ry, int npat, double rmax,
                                int32_t *__restrict__ flag) {
    const int lane = threadIdx.x;
    const int k = blockIdx.x;
    const int b = leaves[k];
    const int s0 = b0[b], cnt = b1[b] - s0;
    if (cnt != npat) {
        if (lane == 0) flag[b] = 0;
        return;
    }
    const double h = side[level[b]];
    const double tol = PATTERN_ULPS * 0x1p-52 * (rmax / h + 1.0);
    bool ok = true;
    for (int j = lane; j < npat; j += 64) {
        const double ex = (px[s0 + j] - cx[b]) / h - rx[j];
        const double ey = (py[s0 + j] - cy[b]) / h - ry[j];
        ok = ok && fabs(ex) <= tol && fabs(ey) <= tol;
    }
    const uint64_t all = __ballot(ok);
    if (lane == 0) flag[b] = (all == ~0ull) ? 1 : 0;
}

template <class T>
static T *upload(vp_plan_s *P, const std::vector<T> &h) {
    T *d = P->mem.alloc<T>(h.size());
    if (!h.empty()) VP_HIP(hipMemcpyAsync(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, P->stream));
    return d;
}

__global__ void k_gather_idx_f64(const double *__restrict__ in, const int32_t *__restrict__ idx,
                                 double *__restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[idx[i]];
}

void build_p2p_gather(vp_plan_s *P, const std::vector<int32_t> &leaves, const std::vector<int32_t> &uptr,
                      const std::vector<int32_t> &uidx, const std::vector<int32_t> &sb, const std::vector<int32_t> &se,
                      const double *sx, const double *sy, P2PGather &g) {
    std::vector<int64_t> ptr(1, 0);
    ptr.reserve(leaves.size() + 1);
    for (int b : leaves) {
        int64_t c = 0;
        for (int e = uptr[b]; e < uptr[b + 1]; ++e) c += se[uidx[e]] - sb[uidx[e]];
        ptr.push_back(ptr.back() + c);
    }
    std::vector<int32_t> idx((size_t)ptr.back());
    size_t k = 0;
    for (int b : leaves)
        for (int e = uptr[b]; e < uptr[b + 1]; ++e)
            for (int j = sb[uidx[e]]; j < se[uidx[e]]; ++j) idx[k++] = j;
    g.len = ptr.back();
    g.ptr = upload(P, ptr);
    g.idx = upload(P, idx);
    g.x = P->mem.alloc<double>((size_t)std::max<int64_t>(g.len, 1));
    g.y = P->mem.alloc<double>((size_t)std::max<int64_t>(g.len, 1));
    if (g.len > 0) {
        const unsigned blocks = (unsigned)((g.len + 255) / 256);
        hipLaunchKernelGGL(k_gather_idx_f64, dim3(blocks), dim3(256), 0, P->stream, sx, g.idx, g.x, g.len);
        hipLaunchKernelGGL(k_gather_idx_f64, dim3(blocks), dim3(256), 0, P->stream, sy, g.idx, g.y, g.len);
        VP_LAUNCH_CHECK();
    }
    VP_HIP(hipStreamSynchronize(P->stream));  // host vectors leave scope
}

void build_near_tables(vp_plan_s *P) {
    Tree &T = P->tree;
    NearTables &N = P->near;
    hipStream_t s = P->stream;
    const int nbox = T.nbox;
    std::vector<int32_t> lev(nbox), ix(nbox), iy(nbox), sb(nbox), se(nbox), nch(nbox), leaves(T.nleaf);
    std::vector<int32_t> uptr(nbox + 1), uidx(T.llen[0]), wptr(nbox + 1);
    VP_HIP(hipMemcpyAsync(lev.data(), T.level, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(ix.data(), T.ix, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(iy.data(), T.iy, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(sb.data(), T.sb, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(se.data(), T.se, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(nch.data(), T.nchild, 4 * nbox, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(leaves.data(), T.leaves, 4 * T.nleaf, hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(uptr.data(), T.lptr[0], 4 * (nbox + 1), hipMemcpyDeviceToHost, s));
    if (T.llen[0]) VP_HIP(hipMemcpyAsync(uidx.data(), T.lidx[0], 4 * T.llen[0], hipMemcpyDeviceToHost, s));
    VP_HIP(hipMemcpyAsync(wptr.data(), T.lptr[2], 4 * (nbox + 1), hipMemcpyDeviceToHost, s));
    VP_HIP(hipStreamSynchronize(s));

    std::vector<int32_t> flag(nbox, 0);
    int npat = 0;
    std::vector<double> rx, ry;
    const bool want = P->self && P->opt.p2p_mode != VP_P2P_PAIRWISE && T.nlevels >= 1;
    if (want) {
        // most frequent leaf size that the matrix cores can take
        std::map<int, int> hist;
        for (int b : leaves) hist[se[b] - sb[b]]++;
        int best = 0, bestc = 0;
        for (auto &kv : hist)
            if (pattern_op_supported(kv.first, P->PD) && kv.second > bestc) {
                best = kv.first;
                bestc = kv.second;
            }
        if (best > 0 && bestc >= 2) {
            TempArena tmp;
            double *drx = tmp.alloc<double>(best), *dry = tmp.alloc<double>(best);
            int32_t *dflag = tmp.alloc<int32_t>(nbox);
            fill_i32(dflag, 0, nbox, s);
            const double *rt = P->opt.root;
            const double rmax = std::max(std::max(std::fabs(rt[0]), std::fabs(rt[0] + rt[2])),
                                         std::max(std::fabs(rt[1]), std::fabs(rt[1] + rt[2])));
            int tried = 0, best_match = -1;
            std::vector<double> hx(best), hy(best), bx, by;
            for (int b : leaves) {
                if (se[b] - sb[b] != best || tried >= 4) continue;
                ++tried;
                // reference coordinates from this leaf
                double cx, cy;
                VP_HIP(hipMemcpy(hx.data(), P->sx + sb[b], 8 * best, hipMemcpyDeviceToHost));
                VP_HIP(hipMemcpy(hy.data(), P->sy + sb[b], 8 * best, hipMemcpyDeviceToHost));
                VP_HIP(hipMemcpy(&cx, T.cx + b, 8, hipMemcpyDeviceToHost));
                VP_HIP(hipMemcpy(&cy, T.cy + b, 8, hipMemcpyDeviceToHost));
                const double h = T.side[lev[b]];
                for (int j = 0; j < best; ++j) {
                    hx[j] = (hx[j] - cx) / h;
                    hy[j] = (hy[j] - cy) / h;
                }
                VP_HIP(hipMemcpyAsync(drx, hx.data(), 8 * best, hipMemcpyHostToDevice, s));
                VP_HIP(hipMemcpyAsync(dry, hy.data(), 8 * best, hipMemcpyHostToDevice, s));
                hipLaunchKernelGGL(k_match_pattern, dim3(T.nleaf), dim3(64), 0, s, T.leaves, T.nleaf, T.sb, T.se,
                                   P->sx, P->sy, T.cx, T.cy, T.level, T.d_side, drx, dry, best, rmax, dflag);
                VP_LAUNCH_CHECK();
                std::vector<int32_t> hf(nbox);
                VP_HIP(hipMemcpyAsync(hf.data(), dflag, 4 * nbox, hipMemcpyDeviceToHost, s));
                VP_HIP(hipStreamSynchronize(s));
                int cnt = 0;
                for (int v : hf) cnt += v;
                if (cnt > best_match) {
                    best_match = cnt;
                    flag = hf;
                    bx = hx;
                    by = hy;
                }
                if (2 * cnt >= bestc) break;
            }
            if (best_match >= 2) {
                npat = best;
                rx = bx;
                ry = by;
            } else {
                std::fill(flag.begin(), flag.end(), 0);
            }
        }
    }
    N.active = npat > 0;
    N.npat = npat;
    N.pat_rx = rx;
    N.pat_ry = ry;

    // --- U lists split: table slots for pattern-leaf pairs on the same level
    // or one level apart, the rest pairwise.  Slot layout per target level
    // (NTOPS = 41): 0..8 same-level neighbour (dx, dy) in -1..1; 9..24 a coarser
    // leaf (side 2h) whose corner lies at (ox, oy) target widths from the
    // target's corner, ox, oy in -2..1; 25..40 a finer leaf (side h/2) at
    // (ox, oy) half widths, ox, oy in -1..2.
    std::vector<int32_t> tslot((size_t)nbox * NTOPS, -1), rptr(nbox + 1, 0), ridx;
    ridx.reserve(uidx.size());
    std::vector<std::vector<int32_t>> cols_by_level(T.nlevels);
    for (int b = 0; b < nbox; ++b) {
        rptr[b] = (int32_t)ridx.size();
        const bool pt = N.active && nch[b] == 0 && flag[b];
        bool used = false;
        for (int e = uptr[b]; e < uptr[b + 1]; ++e) {
            const int a = uidx[e];
            int o = -1;
            if (pt && flag[a]) {
                if (lev[a] == lev[b]) {
                    o = (iy[a] - iy[b] + 1) * 3 + (ix[a] - ix[b] + 1);
                } else if (lev[a] == lev[b] - 1) {
                    const int ox = 2 * ix[a] - ix[b], oy = 2 * iy[a] - iy[b];
                    if (ox >= -2 && ox <= 1 && oy >= -2 && oy <= 1) o = 9 + (oy + 2) * 4 + (ox + 2);
                } else if (lev[a] == lev[b] + 1) {
                    const int ox = ix[a] - 2 * ix[b], oy = iy[a] - 2 * iy[b];
                    if (ox >= -1 && ox <= 2 && oy >= -1 && oy <= 2) o = 25 + (oy + 1) * 4 + (ox + 1);
                }
            }
            if (o >= 0) {
                tslot[(size_t)b * NTOPS + o] = a;
                used = true;
            } else {
                ridx.push_back(a);
            }
        }
        if (used) cols_by_level[lev[b]].push_back(b);
    }
    rptr[nbox] = (int32_t)ridx.size();
    N.pair_uptr = upload(P, rptr);
    N.pair_uidx = upload(P, ridx);
    N.rest_len = (int64_t)ridx.size();
    std::vector<int32_t> rest_leaves;
    for (int b : leaves)
        if (rptr[b + 1] > rptr[b]) rest_leaves.push_back(b);
    // longest lists first: the most expensive leaves start in the first wave of blocks
    {
        std::vector<int64_t> work(nbox, 0);
        for (int b : rest_leaves)
            for (int e = rptr[b]; e < rptr[b + 1]; ++e) work[b] += (int64_t)(se[b] - sb[b]) * (se[ridx[e]] - sb[ridx[e]]);
        std::stable_sort(rest_leaves.begin(), rest_leaves.end(), [&](int x, int y) { return work[x] > work[y]; });
    }
    N.rest_leaves = upload(P, rest_leaves);
    N.n_rest_leaves = (int)rest_leaves.size();
    if (N.active) {
        build_p2p_gather(P, rest_leaves, rptr, ridx, sb, se, P->sx, P->sy, N.g_rest);
    } else {
        // no tables: the full U lists, with nodes as sources (evaluation) and,
        // for separate targets, targets as sources (adjoint)
        build_p2p_gather(P, leaves, uptr, uidx, sb, se, P->sx, P->sy, P->g_fwd);
    }
    // target ranges: the nodes themselves, or a separate target set
    std::vector<int32_t> tb = sb, te = se;
    if (!P->self) {
        VP_HIP(hipMemcpyAsync(tb.data(), T.tb, 4 * nbox, hipMemcpyDeviceToHost, s));
        VP_HIP(hipMemcpyAsync(te.data(), T.te, 4 * nbox, hipMemcpyDeviceToHost, s));
        VP_HIP(hipStreamSynchronize(s));
        if (!N.active) build_p2p_gather(P, leaves, uptr, uidx, tb, te, P->tx, P->ty, P->g_adj);
    }

    // (target, source) pairs the pairwise kernel evaluates in the forward sum
    int64_t pairs = 0;
    for (int b = 0; b < nbox; ++b)
        for (int e = rptr[b]; e < rptr[b + 1]; ++e) pairs += (int64_t)(te[b] - tb[b]) * (se[ridx[e]] - sb[ridx[e]]);
    P->near_pairs = pairs;
    // (target, source) pairs the near-field tables serve, per density
    int64_t tpairs = 0;
    for (size_t i = 0; i < tslot.size(); ++i)
        if (tslot[i] >= 0) {
            const int b = (int)(i / NTOPS), a = tslot[i];
            tpairs += (int64_t)(se[b] - sb[b]) * (se[a] - sb[a]);
        }
    P->table_pairs = tpairs;

    std::vector<int32_t> ident(nbox);
    for (int b = 0; b < nbox; ++b) ident[b] = b;
    N.ident_slot = upload(P, ident);

    // lists for P2M / L2P / far evaluation
    std::vector<int32_t> p2m_pat, p2m_rest, l2p_pat, far_leaves, local_done(nbox, 0);
    for (int b : leaves) {
        const bool pt = N.active && flag[b];
        if (lev[b] >= 2) (pt ? p2m_pat : p2m_rest).push_back(b);
        if (pt && lev[b] >= 2) {
            l2p_pat.push_back(b);
            local_done[b] = 1;
        }
        if (!(pt && lev[b] >= 2) || wptr[b + 1] > wptr[b]) far_leaves.push_back(b);
    }
    N.l2p_pat = upload(P, l2p_pat);
    N.l2p_rest = upload(P, p2m_rest);  // the non-pattern leaves of level >= 2
    N.n_l2p_rest = (int)p2m_rest.size();
    N.n_l2p_pat = (int)l2p_pat.size();
    std::stable_sort(far_leaves.begin(), far_leaves.end(),
                     [&](int x, int y) { return wptr[x + 1] - wptr[x] > wptr[y + 1] - wptr[y]; });
    N.far_leaves = upload(P, far_leaves);
    N.n_far_leaves = (int)far_leaves.size();
    N.local_done = upload(P, local_done);

    // within a level, order the table leaves by their set of slots (stable):
    // 16-column tiles then share their operators where the tree is not uniform
    for (auto &cl : cols_by_level) {
        auto key = [&](int b) {
            uint64_t m = 0;
            for (int o = 0; o < NTOPS; ++o)
                if (tslot[(size_t)b * NTOPS + o] >= 0) m |= 1ull << o;
            return m;
        };
        std::stable_sort(cl.begin(), cl.end(), [&](int x, int y) { return key(x) < key(y); });
    }
    N.nleaf_tab = 0;
    N.tab_levels.clear();
    N.tab_cols_begin.clear();
    std::vector<int32_t> tcols;
    for (int l = 0; l < T.nlevels; ++l)
        if (!cols_by_level[l].empty()) {
            N.tab_levels.push_back(l);
            N.tab_cols_begin.push_back((int)tcols.size());
            tcols.insert(tcols.end(), cols_by_level[l].begin(), cols_by_level[l].end());
            N.nleaf_tab += (int)cols_by_level[l].size();
        }
    N.tab_cols_begin.push_back((int)tcols.size());
    N.tab_cols = upload(P, tcols);
    {
        // First writers store instead of adding to zeroed sums.  Near field:
        // the tables store the sums of their leaves (one tile covers all of a
        // leaf's slots), so only the other leaves are zeroed before the
        // pairwise kernel adds.  Far field: the pattern L2P stores, or adds
        // where the W lists (evaluated before it) have written; the leaves it
        // does not serve and those with W lists are zeroed first.  When every
        // leaf with targets is a pattern L2P leaf without a W list, the L2P
        // launch also adds the near field and the correction row and writes
        // the output (forward evaluations).
        std::vector<char> in_tab(nbox, 0), in_l2p(nbox, 0);
        for (int b : tcols) in_tab[b] = 1;
        for (int b : l2p_pat) in_l2p[b] = 1;
        std::vector<int32_t> zn, zf, fadd(nbox, 0);
        bool any_w = false;
        for (int b : leaves) {
            if (se[b] <= sb[b]) continue;  // no targets (targets are the nodes here)
            const bool w = wptr[b + 1] > wptr[b];
            if (!in_tab[b]) zn.push_back(b);
            if (!in_l2p[b] || w) zf.push_back(b);
            fadd[b] = w ? 1 : 0;
            any_w = any_w || w;
        }
        N.n_zero_near = (int)zn.size();
        N.n_zero_far = (int)zf.size();
        N.zero_near = upload(P, zn);
        N.zero_far = upload(P, zf);
        N.far_add = any_w ? upload(P, fadd) : nullptr;
        N.fused_finish = N.active && zf.empty() && N.n_l2p_rest == 0 && N.n_l2p_pat > 0;
    }
    {
        // one slot row per box spanning all table levels: the NTOPS slots of
        // the box's own level block hold its table sources, every other slot is -1
        const int nt = (int)N.tab_levels.size();
        std::vector<int32_t> lvl_block(T.nlevels, -1);
        for (int li = 0; li < nt; ++li) lvl_block[N.tab_levels[li]] = li;
        const size_t wrow = (size_t)NTOPS * std::max(nt, 1);
        std::vector<int32_t> wide((size_t)nbox * wrow, -1);
        for (int b = 0; b < nbox; ++b) {
            const int li = lvl_block[lev[b]];
            if (li < 0) continue;
            for (int o = 0; o < NTOPS; ++o) wide[(size_t)b * wrow + (size_t)li * NTOPS + o] = tslot[(size_t)b * NTOPS + o];
        }
        N.tab_slot = upload(P, wide);
        // operators present per group of W (table leaf, density) columns:
        // 16-column tiles, and 32-column pairs of tiles for the one-wave form
        const int64_t ncols = (int64_t)tcols.size() * P->nbatch;
        std::vector<char> seen(wrow);
        auto groups = [&](int64_t W, int32_t *&dptr, int32_t *&dops, int32_t *&dorder) {
            std::vector<int32_t> tptr(1, 0), tops;
            for (int64_t t = 0; t * W < ncols; ++t) {
                std::fill(seen.begin(), seen.end(), 0);
                for (int64_t c = W * t; c < std::min(ncols, W * t + W); ++c) {
                    const int b = tcols[c / P->nbatch];
                    for (size_t o = 0; o < wrow; ++o)
                        if (wide[(size_t)b * wrow + o] >= 0) seen[o] = 1;
                }
                for (size_t o = 0; o < wrow; ++o)
                    if (seen[o]) tops.push_back((int32_t)o);
                tptr.push_back((int32_t)tops.size());
            }
            dptr = upload(P, tptr);
            dops = upload(P, tops);
            dorder = upload(P, tile_order_by_work(tptr));
            VP_HIP(hipStreamSynchronize(s));  // the host vectors leave scope
            return (int64_t)tops.size();
        };
        N.table_tile_ops = groups(16, N.tile_ptr, N.tile_ops, N.tile_order);
        groups(32, N.tile2_ptr, N.tile2_ops, N.tile2_order);
    }

    if (N.active) {
        const int np = npat;
        // near-field matrices per target level and slot, A-fragment order
        // (rows = targets, cols = sources).  In units of the target side h a
        // source j sits at c + m xi_j relative to the target centre, target i
        // at xi_i: same level m = 1, c = (dx, dy); coarser m = 2,
        // c = (ox + 1/2, oy + 1/2); finer m = 1/2, c = ((ox - 1/2)/2, (oy - 1/2)/2).
        std::vector<double> K((size_t)N.tab_levels.size() * NTOPS * np * np, 0.0), R((size_t)np * np);
        for (size_t li = 0; li < N.tab_levels.size(); ++li) {
            const double h = T.side[N.tab_levels[li]];
            const double two_log_h = 2.0 * std::log(h);
            for (int o = 0; o < NTOPS; ++o) {
                double cxo, cyo, m;
                if (o < 9) {
                    cxo = (o % 3) - 1;
                    cyo = (o / 3) - 1;
                    m = 1.0;
                } else if (o < 25) {
                    cxo = ((o - 9) % 4 - 2) + 0.5;
                    cyo = ((o - 9) / 4 - 2) + 0.5;
                    m = 2.0;
                } else {
                    cxo = (((o - 25) % 4 - 1) - 0.5) * 0.5;
                    cyo = (((o - 25) / 4 - 1) - 0.5) * 0.5;
                    m = 0.5;
                }
                for (int i = 0; i < np; ++i)
                    for (int j = 0; j < np; ++j) {
                        const double ex = cxo + m * rx[j] - rx[i], ey = cyo + m * ry[j] - ry[i];
                        const double r2 = ex * ex + ey * ey;
                        R[(size_t)i * np + j] = (r2 == 0.0) ? 0.0 : -INV_4PI * (std::log(r2) + two_log_h);
                    }
                vp_to_frag(R.data(), np, np, np, K.data() + ((size_t)li * NTOPS + o) * np * np);
            }
        }
        N.K = upload(P, K);
        // P2M of a pattern leaf: rows = expansion (PD), cols = pattern points;
        // operator 0 about the leaf centre at its scale, operators 1 + qd about
        // the centre of quadrant qd at half the scale over that quadrant's
        // points (the virtual children of an X-list source leaf)
        const int Pn = P->P, PD = P->PD;
        std::vector<double> A((size_t)PD * np), Af((size_t)5 * PD * np);
        for (int op = 0; op < 5; ++op) {
            std::fill(A.begin(), A.end(), 0.0);
            const int qd = op - 1;
            const double dx = op == 0 ? 0.0 : ((qd & 1) ? 0.25 : -0.25);
            const double dy = op == 0 ? 0.0 : ((qd & 2) ? 0.25 : -0.25);
            const double sc = op == 0 ? 1.0 : 2.0;
            for (int j = 0; j < np; ++j) {
                if (op > 0 && ((rx[j] > 0.0 ? 1 : 0) | (ry[j] > 0.0 ? 2 : 0)) != qd) continue;
                std::complex<double> w(sc * (rx[j] - dx), sc * (ry[j] - dy)), pw(1.0, 0.0);
                A[(size_t)0 * np + j] = 1.0;
                for (int k = 1; k < Pn; ++k) {
                    pw *= w;
                    A[(size_t)k * np + j] = -pw.real() / k;
                    A[(size_t)(Pn + k) * np + j] = -pw.imag() / k;
                }
            }
            vp_to_frag(A.data(), PD, np, np, Af.data() + (size_t)op * PD * np);
        }
        // L2P of a pattern leaf: rows = pattern points, cols = expansion (PD)
        std::vector<double> B((size_t)np * PD, 0.0), Bf((size_t)np * PD);
        for (int i = 0; i < np; ++i) {
            std::complex<double> w(rx[i], ry[i]), pw(1.0, 0.0);
            for (int l = 0; l < Pn; ++l) {
                B[(size_t)i * PD + l] = -INV_2PI * pw.real();
                B[(size_t)i * PD + Pn + l] = INV_2PI * pw.imag();
                pw *= w;
            }
        }
        vp_to_frag(B.data(), np, PD, PD, Bf.data());
        // The pattern leaves fill the tree's deepest level and no other box sits
        // there (uniform grids), with the fused finish: their L2P can start from
        // the parents' local expansions, the L2L into that level folded into
        // one matrix per child class q, B_q = L2P x L2L_q, and forward
        // evaluations skip that L2L launch.  L2L_q as in the scaled form of
        // the translations (t = child offset / parent side = (+-1/4, +-1/4)):
        // B'_l = 2^-l t^-l sum_{k >= l} C(k, l) t^k B_k.
        N.par_l2p = false;
        // (the fused launch addresses the near sums and the output by 32-bit offsets)
        if (!P->fp32 && N.fused_finish && P->nbatch % 16 == 0 && !l2p_pat.empty() &&
            32 * (int64_t)std::max(P->n, P->m) < ((int64_t)1 << 32)) {
            const int Lf = lev[l2p_pat[0]];
            bool ok = Lf >= 3 && Lf == T.nlevels - 1;
            for (int b : l2p_pat) ok = ok && lev[b] == Lf;
            int at_lf = 0;
            for (int b = 0; b < nbox; ++b) at_lf += lev[b] == Lf ? 1 : 0;
            ok = ok && at_lf == (int)l2p_pat.size();
            if (ok) {
                std::vector<int32_t> par(nbox);
                VP_HIP(hipMemcpyAsync(par.data(), T.parent, 4 * nbox, hipMemcpyDeviceToHost, s));
                VP_HIP(hipStreamSynchronize(s));
                std::vector<std::vector<long double>> Cb(Pn, std::vector<long double>(Pn, 0.0L));
                for (int k = 0; k < Pn; ++k) {
                    Cb[k][0] = 1.0L;
                    for (int l = 1; l <= k; ++l) Cb[k][l] = Cb[k - 1][l - 1] + (l < k ? Cb[k - 1][l] : 0.0L);
                }
                std::vector<double> Tq((size_t)PD * PD), Bq((size_t)np * PD), Bqf((size_t)4 * np * PD),
                    Bk((size_t)np * PD);
                vp_to_frag_kmajor(B.data(), np, PD, PD, Bk.data());
                for (int q = 0; q < 4; ++q) {
                    const std::complex<long double> t(0.25L * ((q & 1) ? 1 : -1), 0.25L * ((q >> 1) ? 1 : -1));
                    std::fill(Tq.begin(), Tq.end(), 0.0);
                    for (int j = 0; j < 2 * Pn; ++j) {
                        // input column j: B_k = 1 (j = k) or i (j = Pn + k)
                        const int k = j < Pn ? j : j - Pn;
                        const std::complex<long double> bk = j < Pn ? std::complex<long double>(1, 0)
                                                                    : std::complex<long double>(0, 1);
                        const std::complex<long double> tk = std::pow(t, k);
                        for (int l = 0; l <= k; ++l) {
                            const std::complex<long double> v =
                                std::pow(0.5L, l) * std::pow(t, -l) * Cb[k][l] * tk * bk;
                            Tq[(size_t)l * PD + j] = (double)v.real();
                            Tq[(size_t)(Pn + l) * PD + j] = (double)v.imag();
                        }
                    }
                    for (int i = 0; i < np; ++i)
                        for (int j = 0; j < PD; ++j) {
                            long double acc = 0.0L;
                            for (int r = 0; r < PD; ++r) acc += (long double)B[(size_t)i * PD + r] * Tq[(size_t)r * PD + j];
                            Bq[(size_t)i * PD + j] = (double)acc;
                        }
                    vp_to_frag_kmajor(Bq.data(), np, PD, PD, Bqf.data() + (size_t)q * np * PD);
                }
                // the tiles (box, 16 densities) grouped by child class: a
                // workgroup of the fused launch serves one class
                std::vector<int32_t> rec;
                for (int q = 0; q < 4; ++q) {
                    N.l2p_qbeg[q] = (int)(rec.size() / 4);
                    for (int b : l2p_pat) {
                        const int cq = (ix[b] & 1) | ((iy[b] & 1) << 1);
                        if (cq != q) continue;
                        for (int d = 0; d < P->nbatch; d += 16) rec.insert(rec.end(), {b, par[b] * 4 + cq, d, 0});
                    }
                }
                N.l2p_qbeg[4] = (int)(rec.size() / 4);
                N.l2p_km = upload(P, Bk);
                N.par_km = upload(P, Bqf);
                N.l2p_rec = upload(P, rec);
                N.par_l2p = true;
                N.par_level = Lf;
                VP_HIP(hipStreamSynchronize(s));  // Bk, Bqf, rec leave scope
            }
        }
        // Own-cell corrections folded into the near tables (forward).  On a
        // grid of congruent boxes whose corrections are one shared block A
        // (Section 4: the correction depends on the box shape only), every
        // leaf is one cell, and a leaf's sorted node i is row sigma(i) and
        // column tau(i) of its cell with the same sigma, tau and weights w in
        // every leaf, the correction C f of the leaf equals (A' W^-1)(W f)
        // with A'_ij = A_sigma(i),tau(j): the self slot's operator becomes
        // K_self + A' W^-1 and the correction pass is dropped.  K_self W + A'
        // is the leaf's exact own-cell quadrature matrix (the correction is
        // its difference from the smooth rule, Section 4.1).
        N.corr_folded = false;
        std::vector<int32_t> self_leaves;  // leaves whose own box is a table slot
        for (int b : leaves)
            if (tslot[(size_t)b * NTOPS + 4] == b) self_leaves.push_back(b);
        if (N.fused_finish && P->self && !P->corr_block.empty() && P->opt.kernel != VP_KERNEL_YUKAWA &&
            N.tab_levels.size() == 1 && np == 64 && P->corr_cell_col.size() == self_leaves.size() &&
            P->m == P->n) {
            const std::vector<int32_t> &crow = P->corr_cell_row, &ccol = P->corr_cell_col;
            const int nc = (int)ccol.size();
            std::vector<int32_t> perm(P->n);
            std::vector<double> wu(P->n);
            VP_HIP(hipMemcpyAsync(perm.data(), P->sperm, 4 * (size_t)P->n, hipMemcpyDeviceToHost, s));
            VP_HIP(hipMemcpyAsync(wu.data(), P->w_user, 8 * (size_t)P->n, hipMemcpyDeviceToHost, s));
            VP_HIP(hipStreamSynchronize(s));
            std::vector<int32_t> cell_of(P->m, -1), used(nc, 0);
            bool ok = (int64_t)crow.back() == P->m;
            for (int k = 0; ok && k < nc; ++k) {
                ok = crow[k + 1] - crow[k] == 64 && ccol[k] >= 0 && (int64_t)ccol[k] + 64 <= P->n;
                for (int r = crow[k]; ok && r < crow[k + 1]; ++r) cell_of[r] = k;
            }
            std::vector<int32_t> sig(64), tau(64);
            std::vector<double> wref(64);
            bool first = true;
            for (size_t li = 0; ok && li < self_leaves.size(); ++li) {
                const int b = self_leaves[li];
                ok = se[b] - sb[b] == 64 && lev[b] == N.tab_levels[0];
                const int k = ok ? cell_of[perm[sb[b]]] : -1;
                ok = ok && k >= 0 && !used[k];
                if (!ok) break;
                used[k] = 1;
                for (int i = 0; ok && i < 64; ++i) {
                    const int32_t uu = perm[sb[b] + i];
                    const int32_t si = uu - crow[k], ti = uu - ccol[k];
                    ok = cell_of[uu] == k && ti >= 0 && ti < 64;
                    if (!ok) break;
                    if (first) {
                        sig[i] = si;
                        tau[i] = ti;
                        wref[i] = wu[uu];
                        ok = std::isfinite(wref[i]) && wref[i] != 0.0;
                    } else {
                        ok = sig[i] == si && tau[i] == ti &&
                             std::memcmp(&wref[i], &wu[uu], sizeof(double)) == 0;
                    }
                }
                first = false;
            }
            if (ok) {
                const double h = T.side[N.tab_levels[0]];
                const double two_log_h = 2.0 * std::log(h);
                std::vector<double> Rs((size_t)np * np), Kf(K);
                const std::vector<double> &A = P->corr_block;
                for (int i = 0; i < np; ++i)
                    for (int j = 0; j < np; ++j) {
                        const double ex = rx[j] - rx[i], ey = ry[j] - ry[i];
                        const double r2 = ex * ex + ey * ey;
                        const double g = (r2 == 0.0) ? 0.0 : -INV_4PI * (std::log(r2) + two_log_h);
                        Rs[(size_t)i * np + j] = g + A[(size_t)sig[i] * 64 + tau[j]] / wref[j];
                    }
                vp_to_frag(Rs.data(), np, np, np, Kf.data() + (size_t)4 * np * np);
                N.Kf = upload(P, Kf);
                N.corr_folded = true;
                VP_HIP(hipStreamSynchronize(s));  // Kf leaves scope
            }
        }
        if (P->fp32) {
            std::vector<float> af(Af.begin(), Af.end()), bf(Bf.begin(), Bf.end());
            N.p2m_op_f32 = upload(P, af);
            N.l2p_op_f32 = upload(P, bf);
            VP_HIP(hipStreamSynchronize(s));  // af, bf leave scope
        } else {
            N.p2m_op = upload(P, Af);
            N.l2p_op = upload(P, Bf);
        }
        VP_HIP(hipStreamSynchronize(s));  // K, Af, Bf leave scope
    }

    // Virtual children of X-list source leaves that are pattern leaves: the
    // P2M of quadrant qd is the fixed matrix 1 + qd.  The leaf's sorted
    // sources split into its quadrants at the pattern's quadrant boundaries
    // (the source order of every pattern leaf is the reference order); the
    // plan checks this against each leaf's recorded quadrant ranges.  The
    // other leaves and virtual children go to the VALU kernel.
    {
        const int nv = P->n_vleaf;
        std::vector<int32_t> hv(nv), hsplit((size_t)5 * nv), qcols[4], rest_q;
        if (nv > 0) {
            VP_HIP(hipMemcpyAsync(hv.data(), P->vleaf, 4 * (size_t)nv, hipMemcpyDeviceToHost, s));
            VP_HIP(hipMemcpyAsync(hsplit.data(), P->vsplit_s, 4 * hsplit.size(), hipMemcpyDeviceToHost, s));
            VP_HIP(hipStreamSynchronize(s));
        }
        int qb[5] = {0, 0, 0, 0, npat};  // pattern quadrant boundaries
        bool quad_ok = N.active;
        for (int j = 0, prev = 0; quad_ok && j < npat; ++j) {
            const int qd = (rx[j] > 0.0 ? 1 : 0) | (ry[j] > 0.0 ? 2 : 0);
            quad_ok = qd >= prev && std::fabs(rx[j]) > 1e-6 && std::fabs(ry[j]) > 1e-6;
            for (int t = prev + 1; t <= qd; ++t) qb[t] = j;
            prev = qd;
            if (j == npat - 1)
                for (int t = qd + 1; t < 4; ++t) qb[t] = npat;
        }
        const size_t ncol_all = (size_t)nbox + 4 * (size_t)nv;
        std::vector<int32_t> slot, cols(p2m_pat), jobs(p2m_rest);
        if (N.active) {
            slot.assign(ncol_all * 5, -1);
            for (int b : p2m_pat) slot[(size_t)b * 5] = b;
        }
        for (int v = 0; v < nv; ++v) {
            const int a = hv[v];
            bool pat = quad_ok && flag[a];
            for (int qd = 0; pat && qd <= 4; ++qd) pat = hsplit[5 * v + qd] - sb[a] == qb[qd];
            for (int qd = 0; qd < 4; ++qd) {
                if (pat) {
                    const int c = nbox + 4 * v + qd;
                    qcols[qd].push_back(c);
                    slot[(size_t)c * 5 + 1 + qd] = a;
                } else {
                    rest_q.push_back(~(4 * v + qd));
                }
            }
        }
        for (int qd = 0; qd < 4; ++qd) cols.insert(cols.end(), qcols[qd].begin(), qcols[qd].end());
        jobs.insert(jobs.end(), rest_q.begin(), rest_q.end());
        N.n_p2m_cols = N.active ? (int)cols.size() : 0;
        N.n_p2m_leaf_cols = N.active ? (int)p2m_pat.size() : 0;
        if (N.n_p2m_cols > 0) {
            N.p2m_cols = upload(P, cols);
            N.p2m_slot = upload(P, slot);
        }
        N.n_p2m_jobs_rest = (int)jobs.size();
        const std::vector<P2MJob> jd = p2m_job_descs(P, jobs, false);
        N.p2m_jobs_rest = upload(P, jd);
        VP_HIP(hipStreamSynchronize(s));  // host vectors leave scope
    }
    VP_HIP(hipStreamSynchronize(s));
}

}  // namespace vp

// HIP kernels for gfx950 (MI355X): bipartite H*psi, permutations between
// canonical and bipartite order, and the Lanczos vector operations.
//
// Layout: every block Psi_q is row-major [l][r] (left word = row, right word
// = column), blocks back to back.  The left operator H_L therefore combines
// whole contiguous rows (coalesced reads of other rows), the right operator
// H_R gathers inside one row, which is staged in LDS first; this replaces the
// paper's transposition of the blocks before applying left operators.
//
// Every output element is written by exactly one thread with a fixed
// summation order, and every reduction goes through fixed per-item partial
// slots summed in a fixed order, so results do not depend on the launch
// shape or on what else shares the launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "ecut_internal.h"
#include "kernels.h"

namespace ecut {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block sum; result valid in thread 0.  `red` holds one
// double per wave.
__device__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) s += red[w];
    }
    __syncthreads();
    return s;
}

// Result stores.  A vector larger than the last-level cache is streamed past
// it (non-temporal: its lines would only evict the source rows that later
// work still gathers); a smaller one stays cacheable for the next kernel.
// The choice is a compile-time one: with a run-time flag the compiler merges
// the two stores of the branches into one plain store.
template <bool STREAM>
__device__ __forceinline__ void store_result(double *p, double v) {
    if constexpr (STREAM)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

}  // namespace

// Epilogue factors y = xscale H x - zcoef z: from the descriptor, or from
// device memory when the Lanczos driver keeps them there.
__device__ __forceinline__ double2 epi_factors(const double *dscale, double xscale, double zcoef) {
    return dscale ? make_double2(dscale[0], dscale[1]) : make_double2(xscale, zcoef);
}

// ------------------------------------------------------------------------
// Generic row-tile kernel: any cut, sector-changing cross terms, batches of
// problems.  One work item = rows [row0,row1) of one block, staged in LDS
// (STAGE) so the right-operator gathers hit LDS.
// ------------------------------------------------------------------------
template <bool STAGE>
__global__ __launch_bounds__(ROWS_THREADS) void k_rows(const ProblemDev *__restrict__ probs, const ProblemDev single,
                                                       const ItemDev *__restrict__ items, int n_items) {
    extern __shared__ __align__(16) double lds[];
    __shared__ double red[ROWS_THREADS / 64];
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const ItemDev W = items[it];
        if (W.row1 <= W.row0) continue;   // padding of an XCD-dealt list
        const ProblemDev &P = probs ? probs[W.prob] : single;
        const double2 ef = epi_factors(P.dscale, P.xscale, P.zcoef);
        const BlockDev B = P.blocks[W.block];
        const int dR = B.d_r;
        const int nrows = W.row1 - W.row0;
        const int n = nrows * dR;
        const double *__restrict__ xblk = P.x + B.offset;
        const double *__restrict__ xt = xblk + (int64_t)W.row0 * dR;
        if (STAGE) {
            for (int e = threadIdx.x; e < n; e += blockDim.x) lds[e] = xt[e];
            __syncthreads();
        }
        double part = 0.0;
        for (int e = threadIdx.x; e < n; e += blockDim.x) {
            const int lr = e / dR;
            const int r = e - lr * dR;
            const int l = W.row0 + lr;
            const int gl = B.lbase + l, gr = B.rbase + r;
            const uint32_t lw = P.lwords[gl], rw = P.rwords[gr];
            const double *xrow = STAGE ? (lds + lr * dR) : (xt + (int64_t)lr * dR);
            const double xv = xrow[r];
            double dg = P.diag_l[gl] + P.diag_r[gr];
            for (int k = 0; k < P.n_xdiag; ++k) {
                const XDiagDev X = P.xdiag[k];
                double fl = (double)((lw >> X.li) & 1u), fr = (double)((rw >> X.rj) & 1u);
                if (X.li2 >= 0) fl += (double)((lw >> X.li2) & 1u);
                if (X.rj2 >= 0) fr += (double)((rw >> X.rj2) & 1u);
                if (X.spin_form) { fl -= 0.5; fr -= 0.5; }
                dg += X.coef * fl * fr;
            }
            double acc = dg * xv;
            for (int k = P.hr_ptr[gr]; k < P.hr_ptr[gr + 1]; ++k) acc += P.hr_val[k] * xrow[P.hr_col[k]];
            for (int k = P.hl_ptr[gl]; k < P.hl_ptr[gl + 1]; ++k)
                acc += P.hl_val[k] * xblk[(int64_t)P.hl_col[k] * dR + r];
            for (int k = 0; k < P.n_xbond; ++k) {
                const XBondDev X = P.xbond[k];
                int src, lp, rp;
                if ((lw >> X.li) & 1u) {
                    src = X.label ? B.blk_l2minus : B.blk_lminus;
                    lp = P.maps[X.lmap_del + gl];
                    rp = P.maps[X.rmap_ins + gr];
                } else {
                    src = X.label ? B.blk_l2plus : B.blk_lplus;
                    lp = P.maps[X.lmap_ins + gl];
                    rp = P.maps[X.rmap_del + gr];
                }
                if (src >= 0 && lp >= 0 && rp >= 0) {
                    const BlockDev S = P.blocks[src];
                    double c = X.coef;
                    if (X.fermion) {   // (rank << 1) | sign of each side
                        if ((lp ^ rp) & 1) c = -c;
                        lp >>= 1;
                        rp >>= 1;
                    }
                    acc += c * P.x[S.offset + (int64_t)lp * S.d_r + rp];
                }
            }
            double yv = ef.x * acc;
            const int64_t gi = B.offset + (int64_t)l * dR + r;
            if (P.z) yv -= ef.y * P.z[gi];
            P.y[gi] = yv;
            part += xv * yv;
        }
        if (P.partials) {
            const double s = block_sum(part, red);
            if (threadIdx.x == 0) P.partials[W.slot] = s;
        } else if (STAGE) {
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------------
// Hubbard up/down kernel.  One work group owns one row a (up word) at a
// time, persistent over a row list.  Phase 1 (global memory only): the left
// operator H_up as a combination of whole neighbour rows, accumulated in
// registers, while the own row is staged in LDS.  Phase 2 (LDS only): the
// right operator H_dn through the lo/hi split tables, the U n_up n_dn
// diagonal, the Lanczos epilogue and the store.
// ------------------------------------------------------------------------
template <bool UU, bool UT, bool W16>
__global__ __launch_bounds__(HUB_THREADS) void k_hub(const ProblemDev P, const int32_t *__restrict__ rows, int n_rows,
                                                     int n_xcd, int per_xcd) {
    const double2 ef = epi_factors(P.dscale, P.xscale, P.zcoef);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[HUB_THREADS / 64];
    const HubDev &H = P.hub;
    const int dR = P.blocks[0].d_r;
    const int h = H.h;
    const int nlo = 1 << h, nhi = 1 << (H.n_r - h);
    const int ls = H.lo_stride, hs = H.hi_stride;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        unsigned char *p = smem + off;
        off += (bytes + 15) & ~(size_t)15;
        return p;
    };
    double *xs = (double *)carve((size_t)dR * 8);
    uint16_t *ws16 = nullptr;
    uint32_t *ws32 = nullptr;
    if (W16) ws16 = (uint16_t *)carve((size_t)dR * 2);
    else ws32 = (uint32_t *)carve((size_t)dR * 4);
    int32_t *locnt = (int32_t *)carve((size_t)nlo * 4);
    int32_t *loent = (int32_t *)carve((size_t)nlo * ls * 4);
    int32_t *lorank = (int32_t *)carve((size_t)nlo * 4);
    int32_t *hicnt = (int32_t *)carve((size_t)nhi * 4);
    int32_t *hient = (int32_t *)carve((size_t)nhi * hs * 4);
    int32_t *seg = (int32_t *)carve((size_t)nhi * 4);
    double *cf = (double *)carve((size_t)(H.n_coef > 0 ? H.n_coef : 1) * 8);
    double *ut = UU ? nullptr : (double *)carve(3 * 256 * 8);

    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    for (int i = tid; i < dR; i += nt) {
        if (W16) ws16[i] = H.rwords16[i];
        else ws32[i] = H.rwords32[i];
    }
    for (int i = tid; i < nlo; i += nt) { locnt[i] = H.lo_cnt[i]; lorank[i] = H.lo_rank[i]; }
    for (int i = tid; i < nlo * ls; i += nt) loent[i] = H.lo_ent[i];
    for (int i = tid; i < nhi; i += nt) { hicnt[i] = H.hi_cnt[i]; seg[i] = H.seg_off[i]; }
    for (int i = tid; i < nhi * hs; i += nt) hient[i] = H.hi_ent[i];
    for (int i = tid; i < H.n_coef; i += nt) cf[i] = H.coef[i];

    const int xcd = blockIdx.x % n_xcd;
    const int slot = blockIdx.x / n_xcd;
    const int nslot = gridDim.x / n_xcd;
    const double *__restrict__ X = P.x;
    for (int k = slot; k < per_xcd; k += nslot) {
        const int idx = xcd * per_xcd + k;
        if (idx >= n_rows) break;
        const int a = rows[idx];
        const uint32_t aw = P.lwords[a];
        const int p0 = P.hl_ptr[a], p1 = P.hl_ptr[a + 1];
        const double *__restrict__ xa = X + (int64_t)a * dR;
        double acc[HUB_MAXC];
#pragma unroll
        for (int c = 0; c < HUB_MAXC; ++c) acc[c] = 0.0;
        // phase 1: neighbour rows of the left operator (global, coalesced)
        for (int q = p0; q < p1; ++q) {
            const double v = P.hl_val[q];
            const double *__restrict__ xn = X + (int64_t)P.hl_col[q] * dR;
#pragma unroll
            for (int c = 0; c < HUB_MAXC; ++c) {
                const int r = tid + c * HUB_THREADS;
                if (r < dR) acc[c] += v * xn[r];
            }
        }
#pragma unroll
        for (int c = 0; c < HUB_MAXC; ++c) {
            const int r = tid + c * HUB_THREADS;
            if (r < dR) xs[r] = xa[r];
        }
        if (!UU) {
            for (int i = tid; i < 3 * 256; i += nt) {
                const int byte = i >> 8, v = i & 255;
                double s = 0.0;
                for (int b = 0; b < 8; ++b) {
                    const int site = byte * 8 + b;
                    if (site < H.n_r && ((v >> b) & 1) && ((aw >> site) & 1u)) s += H.u[site];
                }
                ut[i] = s;
            }
        }
        __syncthreads();
        // phase 2: right operator in LDS, diagonal, epilogue
        const double dl = P.diag_l[a];
        double part = 0.0;
#pragma unroll
        for (int c = 0; c < HUB_MAXC; ++c) {
            const int r = tid + c * HUB_THREADS;
            if (r < dR) {
                const uint32_t w = W16 ? (uint32_t)ws16[r] : ws32[r];
                const int lo = (int)(w & (uint32_t)(nlo - 1));
                const int hi = (int)(w >> h);
                const double xv = xs[r];
                double dg = dl;
                if (UU) dg += H.u0 * (double)__popc(aw & w);
                else dg += ut[w & 255u] + ut[256 + ((w >> 8) & 255u)] + ut[512 + ((w >> 16) & 255u)];
                double s = dg * xv;
                {
                    const int n = locnt[lo];
                    const int32_t *e = loent + lo * ls;
                    for (int q = 0; q < n; ++q) {
                        const int en = e[q];
                        double v = UT ? H.hop0 : cf[en & 255];
                        if (en & 256) v = -v;
                        s += v * xs[r + (en >> 9)];
                    }
                }
                {
                    const int n = hicnt[hi];
                    const int32_t *e = hient + hi * hs;
                    for (int q = 0; q < n; ++q) {
                        const int en = e[q];
                        double v = UT ? H.hop0 : cf[en & 255];
                        if (en & 256) v = -v;
                        s += v * xs[r + (en >> 9)];
                    }
                }
                for (int q = 0; q < H.n_xb; ++q) {
                    const int lb = H.xb[4 * q], hb = H.xb[4 * q + 1];
                    if (((lo >> lb) & 1) != ((hi >> hb) & 1)) {
                        const int lo2 = lo ^ (1 << lb), hi2 = hi ^ (1 << hb);
                        const int col = seg[hi2] + lorank[lo2];
                        const int par = __popc((uint32_t)lo & ~((2u << lb) - 1u)) + __popc((uint32_t)hi & ((1u << hb) - 1u));
                        double v = UT ? H.hop0 : cf[H.xb[4 * q + 2]];
                        if (par & 1) v = -v;
                        s += v * xs[col];
                    }
                }
                const int64_t gi = (int64_t)a * dR + r;
                double y = ef.x * (acc[c] + s);
                if (P.z) y -= ef.y * P.z[gi];
                P.y[gi] = y;
                part += xv * y;
            }
        }
        if (P.partials) {
            const double s = block_sum(part, red);
            if (tid == 0) P.partials[a] = s;
        } else {
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------------
// Hubbard up/down kernel on class tiles.  A work item is (rows, class): the
// elements of rows [row0, row0+nrows) whose down word has a high part of
// popcount k.  Inside the tile, with T[sr][j] (sr = row * nseg + segment,
// j = low-word rank), a hop inside the low part is a gather along j with
// j-only offsets (kept in registers: each thread keeps one j for the whole
// item), a hop inside the high part is a shift along sr by a per-segment
// offset, so both stay in LDS.  Phase 1 (global): the left operator as a
// combination of neighbour rows restricted to the tile's columns, the
// crossing bonds of the down word (their sources sit in the neighbouring
// classes of the same row) and the staging of the tile.  Phase 2 (LDS): the
// right operator, the diagonal, the Lanczos epilogue and the store.  Tiles
// are at most a few tens of KB, so several work groups share a CU and one's
// LDS phase overlaps another's memory phase.
// ------------------------------------------------------------------------
template <bool UU, bool UT>
__global__ __launch_bounds__(HUB2_THREADS) void k_hub2(const ProblemDev P, const HubItem *__restrict__ items,
                                                       int n_items, int n_xcd, int per_xcd) {
    const double2 ef = epi_factors(P.dscale, P.xscale, P.zcoef);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[HUB2_THREADS / 64];
    const HubDev &H = P.hub;
    const int dR = P.blocks[0].d_r;
    const int h = H.h;
    const int nhi = 1 << (H.n_r - h), nlo = 1 << h;
    const int hs = H.cls_hi_stride, ls = H.cls_lo_stride;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        unsigned char *p = smem + off;
        off += (bytes + 15) & ~(size_t)15;
        return p;
    };
    double *xs = (double *)carve((size_t)H.max_tile * 8);
    int32_t *segcol = (int32_t *)carve((size_t)H.max_nseg * 4);
    int32_t *hiw = (int32_t *)carve((size_t)H.max_nseg * 4);
    int32_t *hicnt = (int32_t *)carve((size_t)H.max_nseg * 4);
    int32_t *hient = (int32_t *)carve((size_t)H.max_nseg * hs * 4);
    int32_t *segoff = (int32_t *)carve((size_t)nhi * 4);
    int32_t *lorank = (int32_t *)carve((size_t)nlo * 4);
    double *cf = (double *)carve((size_t)(H.n_coef > 0 ? H.n_coef : 1) * 8);

    const int tid = threadIdx.x;
    const int NT = blockDim.x;
    for (int i = tid; i < nhi; i += NT) segoff[i] = H.seg_off[i];
    for (int i = tid; i < nlo; i += NT) lorank[i] = H.lo_rank[i];
    for (int i = tid; i < H.n_coef; i += NT) cf[i] = H.coef[i];

    const int xcd = blockIdx.x % n_xcd;
    const int wslot = blockIdx.x / n_xcd;
    const int nslot = gridDim.x / n_xcd;
    const double *__restrict__ X = P.x;
    int loaded = -1;
    for (int k = wslot; k < per_xcd; k += nslot) {
        const int idx = xcd * per_xcd + k;
        if (idx >= n_items) break;
        const HubItem it = items[idx];
        if (it.nrows == 0) continue;
        const int32_t *cd = H.cls + 8 * it.cls;
        const int L = cd[0], nseg = cd[1], seg_base = cd[2], lo_base = cd[3];
        if (it.cls != loaded) {
            __syncthreads();   // previous item's readers of the class tables are done
            for (int i = tid; i < nseg; i += NT) {
                segcol[i] = H.cls_segcol[seg_base + i];
                hiw[i] = H.cls_hiw[seg_base + i];
                hicnt[i] = H.cls_hicnt[seg_base + i];
            }
            for (int i = tid; i < nseg * hs; i += NT) hient[i] = H.cls_hient[seg_base * hs + i];
            loaded = it.cls;
            __syncthreads();
        }
        const int per_pass = NT / L;
        const int p = tid / L;
        const int j = tid - p * L;
        const bool active = p < per_pass;
        const int nsr = it.nrows * nseg;
        const float inv_nseg = 1.0f / (float)nseg;
        int lon = 0;
        int loe[HUB2_LOREG];
        uint32_t lw = 0;
        if (active) {
            lon = H.cls_locnt[lo_base + j];
            lw = (uint32_t)H.cls_low[lo_base + j];
#pragma unroll
            for (int q = 0; q < HUB2_LOREG; ++q) loe[q] = q < lon ? H.cls_loent[(lo_base + j) * ls + q] : 0;
        }
        // phase 1: stage the tile
        for (int sr = p; active && sr < nsr; sr += per_pass) {
            const int r = (int)(((float)sr + 0.5f) * inv_nseg);
            const int s = sr - r * nseg;
            xs[sr * L + j] = X[(int64_t)(it.row0 + r) * dR + segcol[s] + j];
        }
        __syncthreads();
        // phase 2: left operator and crossing bonds from global memory, right
        // operator from LDS, diagonal, epilogue.  Two elements per iteration,
        // and every global load of both is issued before any is consumed.
        double part = 0.0;
        const bool one_row = it.nrows == 1;
        const int uq0 = P.hl_ptr[it.row0], uq1 = P.hl_ptr[it.row0 + 1];
        for (int sr0 = p; active && sr0 < nsr; sr0 += 2 * per_pass) {
            double nb[2][HUB2_NB];
            double xc[2];
            int rowv[2], colv[2], sv[2], nqv[2];
            bool ok[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int sr = sr0 + u * per_pass;
                ok[u] = sr < nsr;
                const int srs = ok[u] ? sr : sr0;
                const int r = (int)(((float)srs + 0.5f) * inv_nseg);
                const int s = srs - r * nseg;
                rowv[u] = it.row0 + r;
                sv[u] = s;
                colv[u] = segcol[s] + j;
                const int q0 = one_row ? uq0 : P.hl_ptr[rowv[u]];
                const int q1 = one_row ? uq1 : P.hl_ptr[rowv[u] + 1];
                nqv[u] = q1 - q0;
#pragma unroll
                for (int q = 0; q < HUB2_NB; ++q)
                    nb[u][q] = (q < nqv[u]) ? X[(int64_t)P.hl_col[q0 + q] * dR + colv[u]] : 0.0;
                // crossing bonds of the down word (sources in the neighbouring classes)
                xc[u] = 0.0;
                const uint32_t hw = (uint32_t)hiw[s];
                for (int q = 0; q < H.n_xb; ++q) {
                    const int lb = H.xb[4 * q], hb = H.xb[4 * q + 1];
                    if (((lw >> lb) ^ (hw >> hb)) & 1u) {
                        const uint32_t lo2 = lw ^ (1u << lb), hi2 = hw ^ (1u << hb);
                        const int col2 = segoff[hi2] + lorank[lo2];
                        const int par = __popc(lw & ~((2u << lb) - 1u)) + __popc(hw & ((1u << hb) - 1u));
                        double v = UT ? H.hop0 : cf[H.xb[4 * q + 2]];
                        if (par & 1) v = -v;
                        xc[u] += v * X[(int64_t)rowv[u] * dR + col2];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (!ok[u]) continue;
                const int sr = sr0 + u * per_pass;
                const int s = sv[u];
                const int row = rowv[u];
                const int q0 = one_row ? uq0 : P.hl_ptr[row];
                double a = 0.0;
#pragma unroll
                for (int q = 0; q < HUB2_NB; ++q)
                    if (q < nqv[u]) a += P.hl_val[q0 + q] * nb[u][q];
                for (int q = HUB2_NB; q < nqv[u]; ++q)
                    a += P.hl_val[q0 + q] * X[(int64_t)P.hl_col[q0 + q] * dR + colv[u]];
                a += xc[u];
                const int e = sr * L + j;
                const double xv = xs[e];
#pragma unroll
                for (int q = 0; q < HUB2_LOREG; ++q) {
                    if (q < lon) {
                        const int en = loe[q];
                        double v = UT ? H.hop0 : cf[en & 255];
                        if (en & 256) v = -v;
                        a += v * xs[e + (en >> 9)];
                    }
                }
                for (int q = HUB2_LOREG; q < lon; ++q) {
                    const int en = H.cls_loent[(lo_base + j) * ls + q];
                    double v = UT ? H.hop0 : cf[en & 255];
                    if (en & 256) v = -v;
                    a += v * xs[e + (en >> 9)];
                }
                {
                    const int n = hicnt[s];
                    const int32_t *hq = hient + s * hs;
                    for (int q = 0; q < n; ++q) {
                        const int en = hq[q];
                        double v = UT ? H.hop0 : cf[en & 255];
                        if (en & 256) v = -v;
                        a += v * xs[e + (en >> 9) * L];
                    }
                }
                const uint32_t aw = P.lwords[row];
                const uint32_t bw = ((uint32_t)hiw[s] << h) | lw;
                double dg = P.diag_l[row];
                if (UU) {
                    dg += H.u0 * (double)__popc(aw & bw);
                } else {
                    uint32_t both = aw & bw;
                    while (both) {
                        const int site = __ffs(both) - 1;
                        dg += H.u[site];
                        both &= both - 1u;
                    }
                }
                const int64_t gi = (int64_t)row * dR + colv[u];
                double y = ef.x * (a + dg * xv);
                if (P.z) y -= ef.y * P.z[gi];
                P.y[gi] = y;
                part += xv * y;
            }
        }
        if (P.partials) {
            const double sum = block_sum(part, red);
            if (tid == 0) P.partials[it.slot] = sum;
        } else {
            __syncthreads();
        }
    }
}

// colex rank of a word of at most 16 bits from the two byte tables
__device__ __forceinline__ int rank16(uint32_t w, const int32_t *rl, const int32_t *rh) {
    const uint32_t lo = w & 255u;
    return rl[lo] + rh[(w >> 8) * 9u + (uint32_t)__popc(lo)];
}

// ------------------------------------------------------------------------
// Hubbard up/down cut, whole rows (down words of at most 16 bits, even row
// length).  One work group per row a of Psi[a][b]:
//  - the row is read once with 16-byte loads (column pairs) and staged in LDS;
//  - up-spin hops: the neighbour rows of the left CSR (wave-uniform), read
//    at the same column pairs, two rows in flight per thread;
//  - down-spin hops: for every bond whose two sites hold one particle, the
//    hopped word is ranked with the colex byte tables, the rank mapped to its
//    column (class-major order, table in LDS) and the amplitude read from the
//    staged row; sign (-1)^(particles strictly between the sites);
//  - diagonal U_i n_i,up n_i,dn from the two words;
//  - 16-byte stores of y = xscale H x - zcoef z, one partial <x, y> per row.
// ------------------------------------------------------------------------
// n_xcd == 8: work group b runs on XCD b % 8 and walks the b % 8-th
// contiguous chunk of the row order, so the rows in flight on one XCD are
// neighbours in that order (their shared neighbour rows can hit its L2);
// n_xcd == 1: plain grid stride.
template <int NT, int PP, int NB>
__global__ __launch_bounds__(NT, 4) void k_hubrow(const ProblemDev P, const int32_t *__restrict__ rows, int n_rows,
                                                  int dR, int n_xcd) {
    const double2 ef = epi_factors(P.dscale, P.xscale, P.zcoef);
    extern __shared__ __align__(16) double xs[];
    __shared__ int32_t rl[256];
    __shared__ int32_t rh[256 * 9];
    __shared__ uint32_t bm[HUBROW_MAX_BOND], bb[HUBROW_MAX_BOND];
    __shared__ double bc[HUBROW_MAX_BOND];
    __shared__ double red[NT / 64];
    const HubDev &H = P.hub;
    const int tid = threadIdx.x;
    const int n_bond = H.n_dbond;
    for (int i = tid; i < 256; i += NT) rl[i] = H.rank_lo[i];
    for (int i = tid; i < 256 * 9; i += NT) rh[i] = H.rank_hi[i];
    for (int i = tid; i < n_bond; i += NT) {
        bm[i] = H.dbond_mask[i];
        bb[i] = H.dbond_betw[i];
        bc[i] = H.dbond_coef[i];
    }
    const int np = dR >> 1;
    double2 *xs2 = (double2 *)xs;
    uint16_t *colmap = (uint16_t *)(xs + dR);   // column of each canonical down rank
    for (int i = tid; i < dR; i += NT) colmap[i] = (uint16_t)H.col_of_rank[i];
    const uint32_t *__restrict__ wpairs = (const uint32_t *)H.rwords16;   // two 16-bit words per column pair
    const int xcd = blockIdx.x % n_xcd, slot = blockIdx.x / n_xcd, n_slot = gridDim.x / n_xcd;
    const int per = (n_rows + n_xcd - 1) / n_xcd;
    const int k_end = min(n_rows, (xcd + 1) * per);
    for (int k = xcd * per + slot; k < k_end; k += n_slot) {
        const int a = rows[k];
        const double2 *__restrict__ xr = (const double2 *)(P.x + (int64_t)a * dR);
        double2 acc[PP];
        {
            double2 xv[PP];
#pragma unroll
            for (int m = 0; m < PP; ++m) {
                const int p = tid + m * NT;
                xv[m] = p < np ? xr[p] : make_double2(0.0, 0.0);
                acc[m] = make_double2(0.0, 0.0);
            }
            __syncthreads();   // readers of the previous row are done (and the tables are loaded)
#pragma unroll
            for (int m = 0; m < PP; ++m) {
                const int p = tid + m * NT;
                if (p < np) xs2[p] = xv[m];
            }
        }
        // up-spin hops: whole neighbour rows, NB in flight; each element adds
        // them pair by pair, (c0 v0 + c1 v1), in list order, whatever NB is
        {
            const int q0 = P.hl_ptr[a], q1 = P.hl_ptr[a + 1];
            for (int q = q0; q < q1; q += NB) {
                double c[NB];
                const double2 *__restrict__ nr[NB];
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    const bool has = q + u < q1;
                    c[u] = has ? P.hl_val[q + u] : 0.0;
                    nr[u] = (const double2 *)(P.x + (int64_t)P.hl_col[has ? q + u : q] * dR);
                }
                double2 v[NB][PP];
#pragma unroll
                for (int u = 0; u < NB; ++u)
#pragma unroll
                    for (int m = 0; m < PP; ++m) {
                        const int p = tid + m * NT;
                        v[u][m] = p < np && q + u < q1 ? nr[u][p] : make_double2(0.0, 0.0);
                    }
#pragma unroll
                for (int u = 0; u < NB; u += 2)
#pragma unroll
                    for (int m = 0; m < PP; ++m) {
                        acc[m].x += c[u] * v[u][m].x + c[u + 1] * v[u + 1][m].x;
                        acc[m].y += c[u] * v[u][m].y + c[u + 1] * v[u + 1][m].y;
                    }
            }
        }
        __syncthreads();   // the row is staged
        const uint32_t aw = P.lwords[a];
        double part = 0.0;
#pragma unroll
        for (int m = 0; m < PP; ++m) {
            const int p = tid + m * NT;
            if (p >= np) continue;
            const uint32_t wp = wpairs[p];
            double yv[2], x0[2];
            const double2 xx = xs2[p];
            x0[0] = xx.x;
            x0[1] = xx.y;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const uint32_t w = e ? (wp >> 16) : (wp & 0xffffu);
                double d = 0.0;
                for (int b = 0; b < n_bond; ++b) {
                    const uint32_t msk = bm[b];
                    if (__popc(w & msk) != 1) continue;
                    const double v = xs[colmap[rank16(w ^ msk, rl, rh)]];
                    d += (__popc(w & bb[b]) & 1) ? -bc[b] * v : bc[b] * v;
                }
                double dg;
                if (H.uniform_u) {
                    dg = H.u0 * (double)__popc(aw & w);
                } else {
                    dg = 0.0;
                    uint32_t both = aw & w;
                    while (both) {
                        dg += H.u[__ffs(both) - 1];
                        both &= both - 1u;
                    }
                }
                yv[e] = ef.x * ((e ? acc[m].y : acc[m].x) + d + dg * x0[e]);
            }
            const int64_t gp = (int64_t)a * np + p;
            if (P.z) {
                const double2 zz = ((const double2 *)P.z)[gp];
                yv[0] -= ef.y * zz.x;
                yv[1] -= ef.y * zz.y;
            }
            ((double2 *)P.y)[gp] = make_double2(yv[0], yv[1]);
            part += x0[0] * yv[0] + x0[1] * yv[1];
        }
        if (P.partials) {
            const double sum = block_sum(part, red);
            if (tid == 0) P.partials[a] = sum;
        }
    }
}

hipError_t launch_hubrow(const ecut_sectors *s, const ProblemDev &prob, const int32_t *rows_d, int n_rows, int grid,
                         int n_xcd, int threads, int n_cu, hipStream_t st) {
    const int dR = s->blocks[0].d_r;
    if (threads != 256 && threads != 512 && threads != 1024) return hipErrorInvalidValue;
    if (dR % 2 != 0 || dR > 2 * HUBROW_P * threads || !prob.hub.rwords16 || !prob.hub.col_of_rank)
        return hipErrorInvalidValue;
    if (n_xcd != 8) n_xcd = 1;
    // the staged row, then the 16-bit rank -> column table
    const size_t lds = (size_t)dR * 8 + (size_t)dR * 2;
    // rows that fit half the pairs per thread keep four neighbour rows in flight
    const bool short_rows = threads == 512 && dR <= 2 * HUBROW_P_SHORT * 512;
    const void *fn = threads == 256   ? (const void *)k_hubrow<256, HUBROW_P, 2>
                     : short_rows     ? (const void *)k_hubrow<512, HUBROW_P_SHORT, 4>
                     : threads == 512 ? (const void *)k_hubrow<512, HUBROW_P, 2>
                                      : (const void *)k_hubrow<1024, HUBROW_P, 2>;
    if (grid <= 0) {
        int per_cu = 0;
        const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
        if (e != hipSuccess) return e;
        grid = std::max(1, per_cu) * n_cu;
    }
    grid = std::max(n_xcd, (grid / n_xcd) * n_xcd);
    if (threads == 256)
        hipLaunchKernelGGL((k_hubrow<256, HUBROW_P, 2>), dim3(grid), dim3(256), lds, st, prob, rows_d, n_rows, dR, n_xcd);
    else if (short_rows)
        hipLaunchKernelGGL((k_hubrow<512, HUBROW_P_SHORT, 4>), dim3(grid), dim3(512), lds, st, prob, rows_d, n_rows, dR,
                           n_xcd);
    else if (threads == 512)
        hipLaunchKernelGGL((k_hubrow<512, HUBROW_P, 2>), dim3(grid), dim3(512), lds, st, prob, rows_d, n_rows, dR, n_xcd);
    else
        hipLaunchKernelGGL((k_hubrow<1024, HUBROW_P, 2>), dim3(grid), dim3(1024), lds, st, prob, rows_d, n_rows, dR,
                           n_xcd);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Spin blocks of a spatial cut, both parts at most 16 sites.  One work group
// per row tile (rows [row0, row1) of one block); the tile is staged in LDS.
//  - right operator: for each flip-flop term inside the right part whose two
//    spins differ, the flipped word is ranked with two byte-table lookups
//    (colex rank) and the amplitude is gathered from the staged tile;
//  - left operator: whole neighbour rows of the same block, read at the
//    tile's columns (one-row tiles: wave-uniform CSR, SPIN_M loads in flight
//    per thread and neighbour);
//  - cross-cut flip-flops S+_i S-_j + h.c. (Eq. (2), the L_m (x) R_m terms):
//    the source row in the neighbouring block comes from the left map, the
//    source column from ranking the flipped right word;
//  - diagonal: left and right diagonals plus the Jz Sz_i Sz_j cut terms.
// Epilogue as k_rows: y = xscale H x - zcoef z, per-item partial of <x, y>.
// ------------------------------------------------------------------------

// One-row item: every per-row quantity (left word, left CSR, source rows of
// the cross terms) is uniform across the work group.  One LDS buffer: it
// first holds the source rows of the cross terms (one per left site), then
// the item's own row for the right operator.
// LEFT: the left operator here; otherwise its sum is already in y (the
// two-pass kernels' left pass) and is read as the starting value.
// tabR / tabX (given exactly when !LEFT, the two-pass right kernel): the
// block's source-column tables of the right flip-flop terms and the cross
// terms, instead of ranking the flipped words (fermion cut: the column,
// 0xffff for no term; spin cut: the column's byte offset in xs, 8 * dR, the
// zero slot, for no term, and for a cross term the source row's zero slot
// minus the column's byte offset); the terms are summed in the same order
// either way.
// FERM: the spatial Hubbard cut's cross terms (block by the mode's spin,
// fermion signs from the maps and the tables' bit 15) and right hops with
// signs; spin problems compile without them.
static_assert(XTAB_SLOTS >= (1 << XR_MAX), "a table entry for every pattern of the folded sites");

// the staged element at byte offset off of xs (a spin cut's table entry)
__device__ __forceinline__ double lds_at(const double *xs, uint32_t off) {
    return *(const double *)((const char *)xs + off);
}

template <int NT, int M, bool LEFT, bool FERM = false>
__device__ __forceinline__ void spin_one_row(const ProblemDev &P, const BlockDev &B, const ItemDev &W, double *xs,
                                             const int32_t *rl, const int32_t *rh, const uint32_t *fm,
                                             const double *fc, int n_flip, double *red, double *xtab,
                                             const uint16_t *__restrict__ tabR = nullptr,
                                             const uint16_t *__restrict__ tabX = nullptr) {
    const double2 ef = epi_factors(P.dscale, P.xscale, P.zcoef);
    const int tid = threadIdx.x;
    const int dR = B.d_r;
    const int l = W.row0;
    const int gl = B.lbase + l;
    const uint32_t lw = P.lwords[gl];
    const double *__restrict__ xblk = P.x + B.offset;
    const double *__restrict__ xt = xblk + (int64_t)l * dR;
    double acc[M];
    uint32_t wr[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int e = tid + m * NT;
        wr[m] = e < dR ? P.rwords[B.rbase + e] : 0u;
        acc[m] = 0.0;
    }
    if (!LEFT) {
        double *__restrict__ yt = P.y + B.offset + (int64_t)l * dR;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int e = tid + m * NT;
            acc[m] = e < dR ? yt[e] : 0.0;
        }
    }
    // left operator: neighbour rows of the same block at the same columns
    if (LEFT) {
        const int q1 = P.hl_ptr[gl + 1];
        for (int q = P.hl_ptr[gl]; q < q1; ++q) {
            const double c = P.hl_val[q];
            const double *__restrict__ xn = xblk + (int64_t)P.hl_col[q] * dR;
            double v[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int e = tid + m * NT;
                v[m] = e < dR ? xn[e] : 0.0;
            }
#pragma unroll
            for (int m = 0; m < M; ++m) acc[m] += c * v[m];
        }
    }
    // cross-cut flip-flops, grouped by left site: the source row (one per
    // left site) is staged in xs, then every bond of the group gathers from it
    const int nx = P.n_xbond;
    int k = 0;
    while (k < nx) {
        const int li = P.xbond[k].li;
        int k1 = k + 1;
        while (k1 < nx && P.xbond[k1].li == li) ++k1;
        const uint32_t bl = (lw >> li) & 1u;
        // the block with one particle of this mode's kind more or fewer on the left
        int src;
        if constexpr (FERM)
            src = P.xbond[k].label ? (bl ? B.blk_l2minus : B.blk_l2plus) : (bl ? B.blk_lminus : B.blk_lplus);
        else
            src = bl ? B.blk_lminus : B.blk_lplus;
        int lp = src >= 0 ? P.maps[(bl ? P.xbond[k].lmap_del : P.xbond[k].lmap_ins) + gl] : -1;
        bool lneg = false;   // fermions: the left part's sign, in the map's low bit
        if (FERM && lp >= 0) {
            lneg = lp & 1;
            lp >>= 1;
        }
        if (lp >= 0) {
            const BlockDev S = P.blocks[src];
            const double *__restrict__ srow = P.x + S.offset + (int64_t)lp * S.d_r;
            // every row of a problem on this kernel fits NT * M elements; all
            // loads of the row are in flight before the barrier
            double sv[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int e = tid + m * NT;
                sv[m] = e < S.d_r ? srow[e] : 0.0;
            }
            __syncthreads();   // earlier readers of xs are done
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int e = tid + m * NT;
                if (e < S.d_r) xs[e] = sv[m];
            }
            if (!FERM && !LEFT && tid == 0) xs[S.d_r] = 0.0;   // the slot a term that does not apply reads
            __syncthreads();
            const uint32_t flipm = bl ? ~0u : 0u;   // bit rj of w ^ flipm: the term applies
            const int32_t zs = 8 * S.d_r;            // the zero slot's byte offset
            for (int kk = k; kk < k1; ++kk) {
                const int rj = P.xbond[kk].rj;
                const double c = lneg ? -P.xbond[kk].coef : P.xbond[kk].coef;
                if constexpr (!LEFT) {   // from the table
                    uint32_t sx[M];
#pragma unroll
                    for (int m = 0; m < M; ++m) {
                        const int e = tid + m * NT;
                        sx[m] = e < dR ? tabX[(int64_t)kk * dR + e] : 0u;
                    }
                    if constexpr (FERM) {
#pragma unroll
                        for (int m = 0; m < M; ++m) {
                            const int e = tid + m * NT;
                            if (e < dR && ((wr[m] >> rj) & 1u) != bl)
                                acc[m] += (sx[m] & 0x8000u ? -c : c) * xs[sx[m] & 0x7fffu];
                        }
                    } else {
                        // branch-free: a term that does not apply adds c * 0 from
                        // the zero slot, so all reads of the bond are in flight
                        // together. The entry is the zero slot minus the source
                        // column (bytes); the sign-extended bit test (-1 where the
                        // term applies, bit rj of the word differing from bl)
                        // scales it. A slot past the row end (sx 0) reads the
                        // zero slot, and its sum is never stored.
                        double v[M];
#pragma unroll
                        for (int m = 0; m < M; ++m) {
                            const int32_t on = __builtin_amdgcn_sbfe((int32_t)(wr[m] ^ flipm), rj, 1);
                            v[m] = lds_at(xs, (uint32_t)(zs + on * (int32_t)sx[m]));
                        }
#pragma unroll
                        for (int m = 0; m < M; ++m) acc[m] += c * v[m];
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < M; ++m) {
                        const int e = tid + m * NT;
                        if (e < dR && ((wr[m] >> rj) & 1u) != bl)
                            acc[m] += c * xs[rank16(wr[m] ^ (1u << rj), rl, rh)];
                    }
                }
            }
        }
        k = k1;
    }
    // the item's own row
    {
        double xv[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int e = tid + m * NT;
            xv[m] = e < dR ? xt[e] : 0.0;
        }
        __syncthreads();   // readers of the last source row are done
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int e = tid + m * NT;
            if (e < dR) xs[e] = xv[m];
        }
        if (!FERM && !LEFT && tid == 0) xs[dR] = 0.0;   // the slot a term that does not apply reads
        if (!LEFT && !FERM && P.n_xr > 0 && tid < (1 << P.n_xr)) {
            // the row's Sz Sz cross terms for every pattern of the n_xr right
            // sites: t = sum_g (bit g ? +1 : -1) xdl[gl][g], in g order
            double t = 0.0;
            for (int g = 0; g < P.n_xr; ++g) {
                const double h = P.xdl[(int64_t)gl * P.n_xr + g];
                t += ((tid >> g) & 1) ? h : -h;
            }
            xtab[tid] = t;
        }
        __syncthreads();
    }
    // right operator from the staged row, diagonal, epilogue
    double dgl = P.diag_l[gl];
    double xh[XR_MAX];   // one pass: the row's folded Sz Sz cross terms
#pragma unroll
    for (int g = 0; g < XR_MAX; ++g) xh[g] = LEFT && !FERM && g < P.n_xr ? P.xdl[(int64_t)gl * P.n_xr + g] : 0.0;
    double part = 0.0;
    double ra[M];
#pragma unroll
    for (int m = 0; m < M; ++m) ra[m] = 0.0;
    if constexpr (!LEFT && FERM) {   // four terms' source columns (and signs) per 8-byte load
        for (int g = 0; g * 4 < n_flip; ++g) {
            uint64_t t[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int e = tid + m * NT;
                t[m] = e < dR ? *(const uint64_t *)(tabR + ((int64_t)g * dR + e) * 4) : ~0ull;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int f = 4 * g + i;
                if (f >= n_flip) break;
                const double cf = fc[f];
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const uint32_t src = (uint32_t)(t[m] >> (16 * i)) & 0xffffu;
                    if (src != 0xffffu) ra[m] += (src & 0x8000u ? -cf : cf) * xs[src & 0x7fffu];
                }
            }
        }
    } else if constexpr (!LEFT) {   // four terms' source columns per 8-byte load
        // branch-free: a spin cut's table holds 8 * dR, the byte offset of the
        // zero slot xs[dR], for "no term" (and in its pads); slots past the
        // row end take four of them
        const uint64_t none4 = (uint64_t)(8u * dR) * 0x0001000100010001ull;
        for (int g = 0; g * 4 < n_flip; ++g) {
            uint64_t t[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int e = tid + m * NT;
                t[m] = e < dR ? *(const uint64_t *)(tabR + ((int64_t)g * dR + e) * 4) : none4;
            }
            double cf[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) cf[i] = 4 * g + i < n_flip ? fc[4 * g + i] : 0.0;
            // per slot: the 4 terms' reads in flight together, then summed in term order
#pragma unroll
            for (int m = 0; m < M; ++m) {
                double v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = lds_at(xs, (uint32_t)(t[m] >> (16 * i)) & 0xffffu);
                // the last word's pad entries are the zero slot's offset and
                // their coefficients 0, so all 4 terms are summed unguarded
#pragma unroll
                for (int i = 0; i < 4; ++i) ra[m] += cf[i] * v[i];
            }
        }
    }
    if constexpr (!LEFT) {
        // the right operator's sum joins acc (the order of the sum is
        // unchanged), and ra takes the diagonal of every slot, all loads in
        // flight together instead of one wait per slot
#pragma unroll
        for (int m = 0; m < M; ++m) acc[m] += ra[m];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int e = tid + m * NT;
            ra[m] = e < dR ? P.diag_r[B.rbase + e] : 0.0;
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int e = tid + m * NT;
        if (e >= dR) continue;
        const uint32_t w = wr[m];
        double a = LEFT ? ra[m] : 0.0;
        if constexpr (LEFT)
            for (int f = 0; f < n_flip; ++f) {
                const uint32_t msk = fm[f];
                if (__popc(w & msk) == 1) a += fc[f] * xs[rank16(w ^ msk, rl, rh)];
            }
        double dg = dgl + (LEFT ? P.diag_r[B.rbase + e] : ra[m]);
        if (!FERM && P.n_xr > 0) {
            if constexpr (LEFT) {   // one pass: the table entry's sum, computed in place
                double t = 0.0;
#pragma unroll
                for (int g = 0; g < XR_MAX; ++g)
                    if (g < P.n_xr) t += ((w >> P.xr_site[g]) & 1u) ? xh[g] : -xh[g];
                dg += t;
            } else {   // the row's table, indexed by the right sites' bits
                uint32_t ix;
                if (P.xr_contig) {
                    ix = (w >> P.xr_lo) & ((1u << P.n_xr) - 1u);
                } else {
                    ix = 0u;
                    for (int g = 0; g < P.n_xr; ++g) ix |= ((w >> P.xr_site[g]) & 1u) << g;
                }
                dg += xtab[ix];
            }
        } else {
            for (int x = 0; x < P.n_xdiag; ++x) {
                const XDiagDev X = P.xdiag[x];
                if constexpr (FERM) {   // densities of the two sites (V n_i n_j)
                    double fl = (double)((lw >> X.li) & 1u), fr = (double)((w >> X.rj) & 1u);
                    if (X.li2 >= 0) fl += (double)((lw >> X.li2) & 1u);
                    if (X.rj2 >= 0) fr += (double)((w >> X.rj2) & 1u);
                    if (X.spin_form) {
                        fl -= 0.5;
                        fr -= 0.5;
                    }
                    dg += X.coef * fl * fr;
                } else {
                    dg += X.coef * ((double)((lw >> X.li) & 1u) - 0.5) * ((double)((w >> X.rj) & 1u) - 0.5);
                }
            }
        }
        const double x0 = xs[e];
        double yv = LEFT ? ef.x * (acc[m] + a + dg * x0) : ef.x * (acc[m] + dg * x0);
        const int64_t gi = B.offset + (int64_t)l * dR + e;
        if (P.z) yv -= ef.y * P.z[gi];
        if constexpr (LEFT) {
            P.y[gi] = yv;
            part += x0 * yv;
        } else {
            acc[m] = yv;
        }
    }
    if constexpr (!LEFT) {
        // the stores after every slot's loads: a wait for a load also waits
        // for the stores issued before it (the memory counter counts both)
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int e = tid + m * NT;
            if (e >= dR) continue;
            P.y[B.offset + (int64_t)l * dR + e] = acc[m];
            part += xs[e] * acc[m];
        }
    }
    if (P.partials) {
        const double sum = block_sum(part, red);
        if (tid == 0) P.partials[W.slot] = sum;
    }
}

// Item of several short rows: per-element rows, cross terms gathered from
// global memory (these blocks are small).
template <int NT, int M, bool LEFT>
__device__ __forceinline__ void spin_many_rows(const ProblemDev &P, const BlockDev &B, const ItemDev &W, double *xs,
                                               const int32_t *rl, const int32_t *rh, const uint32_t *fm,
                                               const double *fc, int n_flip, double *red) {
    const double2 ef = epi_factors(P.dscale, P.xscale, P.zcoef);
    const int tid = threadIdx.x;
    const int dR = B.d_r;
    const int n = (W.row1 - W.row0) * dR;
    const float inv_d = 1.0f / (float)dR;
    const double *__restrict__ xblk = P.x + B.offset;
    const double *__restrict__ xt = xblk + (int64_t)W.row0 * dR;
    // row of element e within the item: (e + 0.5) / dR in single precision is
    // exact after truncation for e, dR < 2^13 (the quotient's rounding error
    // stays below the distance to the next integer)
    auto row_of = [&](int e) { return (int)(((float)e + 0.5f) * inv_d); };
    double acc[M];
    uint32_t wr[M];
    {
        double xv[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int e = tid + m * NT;
            const bool ok = e < n;
            const int lr = row_of(e);
            xv[m] = ok ? xt[e] : 0.0;
            wr[m] = ok ? P.rwords[B.rbase + e - lr * dR] : 0u;
            acc[m] = 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int e = tid + m * NT;
            if (e < n) xs[e] = xv[m];
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int e = tid + m * NT;
        if (e >= n) continue;
        const int lr = row_of(e);
        const int r = e - lr * dR;
        const int gl = B.lbase + W.row0 + lr;
        const uint32_t lw = P.lwords[gl];
        double a = 0.0;
        if (LEFT) {
            const int q1 = P.hl_ptr[gl + 1];
            for (int q = P.hl_ptr[gl]; q < q1; ++q) a += P.hl_val[q] * xblk[(int64_t)P.hl_col[q] * dR + r];
        } else {
            a = P.y[B.offset + (int64_t)W.row0 * dR + e];
        }
        for (int k = 0; k < P.n_xbond; ++k) {
            const XBondDev X = P.xbond[k];
            const uint32_t bl = (lw >> X.li) & 1u;
            if (((wr[m] >> X.rj) & 1u) == bl) continue;
            const int src = bl ? B.blk_lminus : B.blk_lplus;
            if (src < 0) continue;
            const int lp = P.maps[(bl ? X.lmap_del : X.lmap_ins) + gl];
            if (lp < 0) continue;
            const BlockDev S = P.blocks[src];
            a += X.coef * P.x[S.offset + (int64_t)lp * S.d_r + rank16(wr[m] ^ (1u << X.rj), rl, rh)];
        }
        acc[m] = a;
    }
    __syncthreads();
    double part = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
        const int e = tid + m * NT;
        if (e >= n) continue;
        const int lr = row_of(e);
        const int r = e - lr * dR;
        const int gl = B.lbase + W.row0 + lr;
        const uint32_t w = wr[m];
        const uint32_t lw = P.lwords[gl];
        const double *xrow = xs + lr * dR;
        double a = 0.0;
        for (int f = 0; f < n_flip; ++f) {
            const uint32_t msk = fm[f];
            if (__popc(w & msk) == 1) a += fc[f] * xrow[rank16(w ^ msk, rl, rh)];
        }
        double dg = P.diag_l[gl] + P.diag_r[B.rbase + r];
        if (P.n_xr > 0) {   // the folded terms, summed as the one-row kernel's table entry
            double t = 0.0;
            for (int g = 0; g < P.n_xr; ++g) {
                const double h = P.xdl[(int64_t)gl * P.n_xr + g];
                t += ((w >> P.xr_site[g]) & 1u) ? h : -h;
            }
            dg += t;
        } else {
            for (int x = 0; x < P.n_xdiag; ++x) {
                const XDiagDev X = P.xdiag[x];
                dg += X.coef * ((double)((lw >> X.li) & 1u) - 0.5) * ((double)((w >> X.rj) & 1u) - 0.5);
            }
        }
        const double x0 = xs[e];
        double yv = ef.x * (acc[m] + a + dg * x0);
        const int64_t gi = B.offset + (int64_t)W.row0 * dR + e;
        if (P.z) yv -= ef.y * P.z[gi];
        P.y[gi] = yv;
        part += x0 * yv;
    }
    if (P.partials) {
        const double sum = block_sum(part, red);
        if (tid == 0) P.partials[W.slot] = sum;
    }
}

// ONE: items of one row (NT = SPIN_THREADS, M = SPIN_M; xs holds max(d_r)
// doubles: first the cross-term source rows, then the row); otherwise items
// of several short rows (xs holds the tile, at most SPIN_MANY_TILE).  Each
// kernel skips the other kind of item, so both run over the same list.
template <bool ONE>
__global__ __launch_bounds__(ONE ? SPIN_THREADS : SPIN_MANY_THREADS, ONE ? 4 : 2) void k_spin(
    const ProblemDev *__restrict__ probs, const ProblemDev single, const ItemDev *__restrict__ items, int n_items,
    int xtab_off) {
    constexpr int NT = ONE ? SPIN_THREADS : SPIN_MANY_THREADS;
    constexpr int M = ONE ? SPIN_M : SPIN_MANY_TILE / SPIN_MANY_THREADS;
    extern __shared__ __align__(16) double xs[];
    __shared__ double red[NT / 64];
    __shared__ int32_t rl[256];
    __shared__ int32_t rh[256 * 9];
    __shared__ uint32_t fm[SPIN_MAX_FLIP];
    __shared__ double fc[SPIN_MAX_FLIP];
    const int tid = threadIdx.x;
    for (int i = tid; i < 256; i += NT) rl[i] = single.rank_lo[i];
    for (int i = tid; i < 256 * 9; i += NT) rh[i] = single.rank_hi[i];
    int loaded = -1;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
        const ItemDev W = items[it];
        if (W.row1 <= W.row0 || (W.row1 - W.row0 == 1) != ONE) continue;   // padding, or the other kernel's item
        const ProblemDev &P = probs ? probs[W.prob] : single;
        const int n_flip = P.n_rflip;
        if (W.prob != loaded) {
            __syncthreads();
            for (int i = tid; i < n_flip; i += NT) {
                fm[i] = P.rflip_mask[i];
                fc[i] = P.rflip_coef[i];
            }
            loaded = W.prob;
        }
        const BlockDev B = P.blocks[W.block];
        if (ONE)
            spin_one_row<NT, M, true>(P, B, W, xs, rl, rh, fm, fc, n_flip, red, xs + xtab_off);
        else
            spin_many_rows<NT, M, true>(P, B, W, xs, rl, rh, fm, fc, n_flip, red);
    }
}

// ------------------------------------------------------------------------
// Two-pass spin kernels.  Pass 1 (k_spinL): the left operator H_L (x) 1 of
// every block on slab items (64 columns x rows_per_item rows of the block's
// level order), as the Hubbard left pass; y = H_L x.  Pass 2 (k_spinR): the
// one-row and several-row items of the spin kernel without the left
// operator, which start from y; the one-row items come grouped by the
// interior of the left word, so the cross-term source rows of a group (rows
// differing only at the cut's left sites) are read from HBM about once.
// Both passes run one work group per item, dealt to the XCDs in contiguous
// ranges (xcd_item): a group's rows stay on one XCD and in its L2.
// ------------------------------------------------------------------------
__device__ __forceinline__ int xcd_item(int n_xcd, int per_xcd);
template <bool PAIR, bool STREAM, bool OFF32 = false>
__device__ __forceinline__ void hubU_item(const HubUArgs &A, int it);

template <bool STREAM>
__global__ __launch_bounds__(HUBU_THREADS) void k_spinL(const SpinLArgs A, int n_xcd, int per_xcd) {
    const int it = xcd_item(n_xcd, per_xcd);
    if (it >= A.n_items) return;
    int lo = 0, hi = A.n_blocks - 1;   // the last block with item0 <= it
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.blocks[mid].item0 <= it) lo = mid;
        else hi = mid - 1;
    }
    const SpinLBlock L = A.blocks[lo];
    HubUArgs U;
    U.x = A.x + L.offset;
    U.y = A.y + L.offset;
    U.hl_ptr = A.hl_ptr + L.lbase;
    U.hl_col = A.hl_col;
    U.hl_val = A.hl_val;
    U.rows = A.rows + L.lbase;
    U.hop = 0.0;
    U.uniform = 0;
    U.slab_ways = 1;
    U.n_rows = L.d_l;
    U.dR = L.d_r;
    U.rows_per_item = A.rows_per_item;
    U.n_rgroups = L.n_rgroups;
    U.n_slabs = L.n_slabs;
    U.n_items = L.n_rgroups * L.n_slabs;
    hubU_item<false, STREAM>(U, it - L.item0);
}

// ONE: one-row items on NT1 threads with M1 amplitudes each (512 x 13 for
// rows of up to 6,656 amplitudes, 256 x 5 for rows of up to 1,280); the
// source-column tables replace the ranking tables, which only the items of
// several rows (ONE = false) load.
template <bool ONE, int NT1, int M1, bool FERM>
__global__ __launch_bounds__(ONE ? NT1 : SPIN_MANY_THREADS, (ONE && NT1 == SPIN_THREADS) ? 4 : 2) void k_spinR(
    const ProblemDev P, const uint16_t *__restrict__ tab, const int64_t *__restrict__ tbase,
    const ItemDev *__restrict__ items, int n_items, int n_xcd, int per_xcd, int xtab_off) {
    constexpr int NT = ONE ? NT1 : SPIN_MANY_THREADS;
    constexpr int M = ONE ? M1 : SPIN_MANY_TILE / SPIN_MANY_THREADS;
    extern __shared__ __align__(16) double xs[];
    __shared__ double red[NT / 64];
    __shared__ int32_t rl[ONE ? 1 : 256];
    __shared__ int32_t rh[ONE ? 1 : 256 * 9];
    __shared__ uint32_t fm[SPIN_MAX_FLIP];
    __shared__ double fc[SPIN_MAX_FLIP];
    const int it = xcd_item(n_xcd, per_xcd);
    if (it >= n_items) return;   // uniform over the work group
    const ItemDev W = items[it];
    if (W.row1 <= W.row0) return;
    const int tid = threadIdx.x;
    const int n_flip = P.n_rflip;
    if (!ONE) {
        for (int i = tid; i < 256; i += NT) rl[i] = P.rank_lo[i];
        for (int i = tid; i < 256 * 9; i += NT) rh[i] = P.rank_hi[i];
    }
    for (int i = tid; i < n_flip; i += NT) {
        fm[i] = P.rflip_mask[i];
        fc[i] = P.rflip_coef[i];
    }
    __syncthreads();
    const BlockDev B = P.blocks[W.block];
    if constexpr (ONE)
        spin_one_row<NT, M, false, FERM>(P, B, W, xs, rl, rh, fm, fc, n_flip, red, xs + xtab_off, tab + tbase[2 * W.block],
                                         tab + tbase[2 * W.block + 1]);
    else
        spin_many_rows<NT, M, false>(P, B, W, xs, rl, rh, fm, fc, n_flip, red);
}

// ------------------------------------------------------------------------
// Left (up-spin) operator over column slabs: y[a, S] = sum_a' H_up[a,a'] x[a', S]
// for a slab S of SLAB_W consecutive columns.  Every XCD walks a contiguous
// range of slabs, all its work groups on the same slab at the same time (each
// one a chunk of rows), so after the first touch every neighbour-row read of
// the slab is an L2 hit; x is fetched from HBM about once.  Work group w runs
// on XCD w % 8 (round-robin dispatch); per_xcd = gridDim.x / 8.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(SLAB_THREADS) void k_upslab(const double *__restrict__ x, double *__restrict__ y,
                                                         const int32_t *__restrict__ hl_ptr,
                                                         const int32_t *__restrict__ hl_col,
                                                         const double *__restrict__ hl_val, int n_rows, int dR,
                                                         int per_xcd) {
    const int xcd = blockIdx.x % 8;
    const int l = blockIdx.x / 8;
    const int n_slabs = (dR + SLAB_W - 1) / SLAB_W;
    const int spx = (n_slabs + 7) / 8;
    const int rows_per = (n_rows + per_xcd - 1) / per_xcd;
    const int r_begin = l * rows_per;
    const int r_end = min(n_rows, r_begin + rows_per);
    const int lane = threadIdx.x % SLAB_W;
    const int grp = threadIdx.x / SLAB_W;
    const int ngrp = SLAB_THREADS / SLAB_W;
    for (int sl = xcd * spx; sl < min(n_slabs, (xcd + 1) * spx); ++sl) {
        const int c = sl * SLAB_W + lane;
        const bool col_ok = c < dR;
        for (int a = r_begin + grp; a < r_end; a += ngrp) {
            const int q0 = hl_ptr[a], q1 = hl_ptr[a + 1];
            double acc = 0.0;
            int q = q0;
            for (; q + 4 <= q1; q += 4) {
                double v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = col_ok ? x[(int64_t)hl_col[q + u] * dR + c] : 0.0;
#pragma unroll
                for (int u = 0; u < 4; ++u) acc += hl_val[q + u] * v[u];
            }
            for (; q < q1; ++q) acc += hl_val[q] * (col_ok ? x[(int64_t)hl_col[q] * dR + c] : 0.0);
            if (col_ok) y[(int64_t)a * dR + c] = acc;
        }
    }
}

// ------------------------------------------------------------------------
// Fast class-tile kernel for uniform, sign-free hopping (open chains).
// Same items and tiles as k_hub2, but: every hop value is the same -t, so
// all neighbour values are summed first and scaled once; tiles have a row
// stride of L+1 with a zero in the last slot, which unused low-hop entries
// address, so the low-hop gathers are unconditional; the up-spin neighbour
// rows of a one-row item are uniform base pointers, so their loads need no
// per-lane address arithmetic; the crossing bond's source column splits
// into a per-segment and a per-lane part that are both precomputed.
// ------------------------------------------------------------------------
template <bool UP, bool STREAM>
__global__ __launch_bounds__(HUB3_THREADS, HUB3_WAVES_PER_EU) void k_hub3(const Hub3Args A) {
    const double2 ef = epi_factors(A.dscale, A.xscale, A.zcoef);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[HUB3_THREADS / 64];
    const int hs = A.hs;
    double *xs = (double *)smem;
    int4 *sinf = (int4 *)(smem + (((size_t)A.max_tile * 8 + 15) & ~(size_t)15));
    int32_t *hnb = (int32_t *)(sinf + A.max_nseg);
    int32_t *hcnt = hnb + A.max_nseg * hs;
    // the class's per-lane low-hop tables: loinfo, then looff as two int4
    const size_t lo_off = (((size_t)A.max_tile * 8 + 15) & ~(size_t)15) + (size_t)A.max_nseg * 16 +
                          (((size_t)A.max_nseg * hs * 4 + 15) & ~(size_t)15) + (((size_t)A.max_nseg * 4 + 15) & ~(size_t)15);
    int4 *linf = (int4 *)(smem + lo_off);
    int4 *lofs = linf + A.max_l;
    const int tid = threadIdx.x;
    const int NT = blockDim.x;
    const int dR = A.dR;
    const int xcd = blockIdx.x % A.n_xcd;
    const int wslot = blockIdx.x / A.n_xcd;
    const int nslot = gridDim.x / A.n_xcd;
    int loaded = -1;
    for (int k = wslot; k < A.per_xcd; k += nslot) {
        const int idx = xcd * A.per_xcd + k;
        if (idx >= A.n_items) break;
        const HubItem it = A.items[idx];
        if (it.nrows == 0) continue;
        const int32_t *cd = A.cls + 8 * it.cls;
        const int L = cd[0], nseg = cd[1], seg_base = cd[2], lo_base = cd[3];
        if (it.cls != loaded) {
            __syncthreads();
            for (int i = tid; i < nseg; i += NT) {
                sinf[i] = A.seginfo[seg_base + i];
                hcnt[i] = A.hcnt[seg_base + i];
            }
            for (int i = tid; i < nseg * hs; i += NT) hnb[i] = A.hnb[seg_base * hs + i];
            for (int i = tid; i < L; i += NT) {
                linf[i] = A.loinfo[lo_base + i];
                const int4 *src = (const int4 *)(A.looff + (size_t)(lo_base + i) * 8);
                lofs[2 * i] = src[0];
                lofs[2 * i + 1] = src[1];
            }
            loaded = it.cls;
            __syncthreads();
        }
        const int Lp = L + 1;
        const int nsr = it.nrows * nseg;
        const float inv_nseg = 1.0f / (float)nseg;
        const int per_pass = NT / L;
        const int p = tid / L;
        const int j = tid - p * L;
        const bool active = p < per_pass;
        const bool one_row = it.nrows == 1;
        // this thread's element slots: (row r, segment s) = sr = p + m * per_pass
        int col_m[HUB3_M];
        double acc[HUB3_M];
#pragma unroll
        for (int m = 0; m < HUB3_M; ++m) {
            const int sr = p + m * per_pass;
            const bool ok = active && sr < nsr;
            int r = 0, s = sr;
            if (!one_row) {
                r = (int)(((float)sr + 0.5f) * inv_nseg);
                s = sr - r * nseg;
            }
            col_m[m] = ok ? (int)((int64_t)r * dR) + sinf[s].x + j : -1;   // element offset from row0, -1 = unused
            acc[m] = 0.0;
        }
        const double *__restrict__ x0row = A.x + (int64_t)it.row0 * dR;
        // fused kernel: the first row's word, in flight with the tile's loads
        const uint32_t aw0_v = UP ? A.lwords[it.row0] : 0u;
        // stage the tile (row stride L+1, zero in the pad slot); every load
        // of a phase is issued before any result is consumed
        {
            double v[HUB3_M];
#pragma unroll
            for (int m = 0; m < HUB3_M; ++m) v[m] = col_m[m] >= 0 ? x0row[col_m[m]] : 0.0;
            // split mode: the up-spin hops' sum is already in y; it is loaded
            // here, so its loads are in flight with the tile's
            if constexpr (!UP) {
#pragma unroll
                for (int m = 0; m < HUB3_M; ++m)
                    acc[m] = col_m[m] >= 0 ? A.y[(int64_t)it.row0 * dR + col_m[m]] : 0.0;
            }
#pragma unroll
            for (int m = 0; m < HUB3_M; ++m)
                if (col_m[m] >= 0) xs[(p + m * per_pass) * Lp + j] = v[m];
            for (int sr = tid; sr < nsr; sr += NT) xs[sr * Lp + L] = 0.0;
        }
        // up-spin hops (fused mode): neighbour rows at the same columns
        if (UP && one_row) {
            const int uq0 = A.hl_ptr[it.row0], uq1 = A.hl_ptr[it.row0 + 1];
            for (int q = uq0; q < uq1; ++q) {
                const double *__restrict__ xn = A.x + (size_t)A.hl_col[q] * (size_t)dR;
                double v[HUB3_M];
#pragma unroll
                for (int m = 0; m < HUB3_M; ++m) v[m] = col_m[m] >= 0 ? xn[col_m[m]] : 0.0;
#pragma unroll
                for (int m = 0; m < HUB3_M; ++m) acc[m] += v[m];
            }
        } else if (UP) {
#pragma unroll
            for (int m = 0; m < HUB3_M; ++m) {
                if (col_m[m] < 0) continue;
                const int r = (int)(((float)(p + m * per_pass) + 0.5f) * inv_nseg);
                const int row = it.row0 + r;
                const int cl = col_m[m] - (int)((int64_t)r * dR);
                const int q1 = A.hl_ptr[row + 1];
                for (int q = A.hl_ptr[row]; q < q1; ++q) acc[m] += A.x[(int64_t)A.hl_col[q] * dR + cl];
            }
        }
        // down-spin bond across the lo/hi split (source in a neighbouring class)
        int4 li = make_int4(0, 0, 2, 0);
        int lof[8];
        if (active) {
            li = linf[j];
            const int4 o0 = lofs[2 * j], o1 = lofs[2 * j + 1];
            lof[0] = o0.x, lof[1] = o0.y, lof[2] = o0.z, lof[3] = o0.w;
            lof[4] = o1.x, lof[5] = o1.y, lof[6] = o1.z, lof[7] = o1.w;
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) lof[q] = 0;
        }
        {
            double v[HUB3_M];
#pragma unroll
            for (int m = 0; m < HUB3_M; ++m) {
                v[m] = 0.0;
                if (col_m[m] >= 0) {
                    const int srm = p + m * per_pass;
                    const int s = one_row ? srm : srm - nseg * (int)(((float)srm + 0.5f) * inv_nseg);
                    const int4 si = sinf[s];
                    if ((li.z ^ si.w) == 1) v[m] = x0row[col_m[m] - si.x - j + si.z + li.y];
                }
            }
            // acc holds unscaled neighbour sums when fused, hop-weighted sums in split mode
#pragma unroll
            for (int m = 0; m < HUB3_M; ++m) acc[m] += UP ? v[m] : A.hop * v[m];
        }
        __syncthreads();
        // down-spin hops inside the tile, diagonal, epilogue. Split mode:
        // every result first (into acc), then the stores, so that no slot's
        // loads wait for an earlier slot's store (the memory counter counts
        // both); the fused kernel, short of registers, stores as it goes.
        // The two item kinds run separate copies of the loop (ONE: a one-row
        // item, whose row word is aw0), so a one-row item's slots load no row
        // word, and no wait for such a load holds back the next slot.
        double part = 0.0;
        // the first row's word (fused kernel: in a scalar register, so that no
        // slot waits on its load, and with it on the previous slot's store)
        const uint32_t aw0 = UP ? __builtin_amdgcn_readfirstlane(aw0_v) : A.lwords[it.row0];
        auto epilogue = [&](auto one_c) {
        constexpr bool ONE = decltype(one_c)::value;
#pragma unroll
        for (int m = 0; m < HUB3_M; ++m) {
            if (col_m[m] < 0) continue;
            const int sr = p + m * per_pass;
            int r = 0, s = sr;
            if (!ONE) {
                r = (int)(((float)sr + 0.5f) * inv_nseg);
                s = sr - r * nseg;
            }
            const int rb = sr * Lp;
            const double x0 = xs[rb + j];
            double dn = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) dn += xs[rb + j + lof[q]];
            const int hc = hcnt[s];
            const int32_t *hq = hnb + s * hs;
            for (int q = 0; q < hc; ++q) dn += xs[rb + (hq[q] - s) * Lp + j];
            const uint32_t aw = ONE ? aw0 : A.lwords[it.row0 + r];
            const uint32_t bw = ((uint32_t)sinf[s].y << A.h) | (uint32_t)li.x;
            const double dg = A.u0 * (double)__popc(aw & bw);
            const int64_t gi = (int64_t)it.row0 * dR + col_m[m];
            double y = UP ? ef.x * (A.hop * (acc[m] + dn) + dg * x0) : ef.x * (acc[m] + A.hop * dn + dg * x0);
            if (A.z) {
                if constexpr (STREAM)   // read once: kept out of the cache like the result
                    y -= ef.y * __builtin_nontemporal_load(A.z + gi);
                else
                    y -= ef.y * A.z[gi];
            }
            if constexpr (UP) {
                store_result<STREAM>(&A.y[gi], y);
                part += x0 * y;
            } else {
                acc[m] = y;
            }
        }
        };
        if (one_row) epilogue(std::true_type{});
        else epilogue(std::false_type{});
        if constexpr (!UP) {
#pragma unroll
            for (int m = 0; m < HUB3_M; ++m) {
                if (col_m[m] < 0) continue;
                const double x0 = xs[(p + m * per_pass) * Lp + j];
                store_result<STREAM>(&A.y[(int64_t)it.row0 * dR + col_m[m]], acc[m]);
                part += x0 * acc[m];
            }
        }
        if (A.partials) {
            const double sum = block_sum(part, red);
            if (tid == 0) A.partials[it.slot] = sum;
        } else {
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------------
// Segment-tile kernel for uniform, sign-free hopping.  A segment is the set
// of words that share the high half; a tile is Psi[a][b] for a in one up
// segment (a contiguous run of rows) and b in one down segment (a contiguous
// run of columns).  Hops inside the low half of either word stay in the tile
// and are read from LDS.  The other hops read global memory:
//  - up high-half hops: the same columns of the neighbour segment's rows;
//  - down high-half hops: the same rows at the neighbour segment's columns;
//  - the bond across the split, for either spin: one gathered element.
// Items come grouped by panel (one up segment x one down class), and the
// panels are dealt to 8 XCD chunks, so all work groups of an XCD work on one
// or two panels at a time: the down high-hop sources are the other tiles of
// the same panel, fetched into that XCD's L2 by their own item.
// ------------------------------------------------------------------------
__global__ __launch_bounds__(HUBSEG_THREADS, 4) void k_hubseg(const HubSegArgs A) {
    const double2 ef = epi_factors(A.dscale, A.xscale, A.zcoef);
    extern __shared__ __align__(16) double xt[];
    __shared__ double red[HUBSEG_THREADS / 64];
    constexpr int M = HUBSEG_M;
    const int tid = threadIdx.x;
    const int dR = A.dR;
    const int xcd = blockIdx.x % A.n_xcd;
    const int wslot = blockIdx.x / A.n_xcd;
    const int nslot = gridDim.x / A.n_xcd;
    for (int k = wslot; k < A.per_xcd; k += nslot) {
        const int idx = xcd * A.per_xcd + k;
        if (idx >= A.n_items) break;
        const HubSegItem it = A.items[idx];
        if (it.useg < 0) continue;
        const int4 U = A.useg[it.useg];   // first row, rows, up low-table base, high hops
        const int32_t *cd = A.cls + 8 * it.cls;
        const int L = cd[0], seg_base = cd[2], lo_base = cd[3];
        const int4 S = A.seginfo[it.dseg];   // first column, high word, crossing column, crossing bit
        const int Lp = L + 1;
        const int per_pass = HUBSEG_THREADS / L;
        const int p = tid / L;
        const int j = tid - p * L;
        const bool active = p < per_pass;
        int4 li = make_int4(0, 0, 2, 0);
        int lof[8];
        if (active) {
            li = A.loinfo[lo_base + j];
#pragma unroll
            for (int q = 0; q < 8; ++q) lof[q] = A.looff[(lo_base + j) * 8 + q];
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q) lof[q] = 0;
        }
        // element (i, j) of the tile lives at offset (U.x + i) * dR + S.x + j
        int off[M];
        double x0[M], acc[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int i = p + m * per_pass;
            off[m] = (active && i < U.y) ? (U.x + i) * dR + S.x + j : -1;
            acc[m] = 0.0;
        }
#pragma unroll
        for (int m = 0; m < M; ++m) x0[m] = off[m] >= 0 ? A.x[off[m]] : 0.0;
        // up high-half hops: row i of the neighbour segment, same column
        for (int q = 0; q < U.w; ++q) {
            const int d = (A.uhnb[it.useg * A.uhs + q] - U.x) * dR;
            double v[M];
#pragma unroll
            for (int m = 0; m < M; ++m) v[m] = off[m] >= 0 ? A.x[off[m] + d] : 0.0;
#pragma unroll
            for (int m = 0; m < M; ++m) acc[m] += v[m];
        }
        // down high-half hops: same row, the neighbour segment's column
        const int nd = A.hcnt[it.dseg];
        for (int q = 0; q < nd; ++q) {
            const int d = A.seginfo[seg_base + A.hnb[it.dseg * A.hs + q]].x - S.x;
            double v[M];
#pragma unroll
            for (int m = 0; m < M; ++m) v[m] = off[m] >= 0 ? A.x[off[m] + d] : 0.0;
#pragma unroll
            for (int m = 0; m < M; ++m) acc[m] += v[m];
        }
        // the bond across the split: up (source row per row), down (source
        // column in the neighbouring class, per column)
        {
            const bool dx = (li.z ^ S.w) == 1;
            const int dd = S.z + li.y - (S.x + j);
            double v[M];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                v[m] = 0.0;
                if (off[m] >= 0) {
                    const int a = U.x + p + m * per_pass;
                    const int r = A.ucross[a];
                    if (r >= 0) v[m] = A.x[off[m] + (r - a) * dR];
                }
            }
#pragma unroll
            for (int m = 0; m < M; ++m) acc[m] += v[m];
#pragma unroll
            for (int m = 0; m < M; ++m) v[m] = (off[m] >= 0 && dx) ? A.x[off[m] + dd] : 0.0;
#pragma unroll
            for (int m = 0; m < M; ++m) acc[m] += v[m];
        }
        // stage the tile (row stride L + 1, zero in the pad column)
        __syncthreads();   // readers of the previous tile are done
#pragma unroll
        for (int m = 0; m < M; ++m)
            if (off[m] >= 0) xt[(p + m * per_pass) * Lp + j] = x0[m];
        for (int r = tid; r < U.y; r += HUBSEG_THREADS) xt[r * Lp + L] = 0.0;
        __syncthreads();
        // low-half hops of both spins from the tile, diagonal, epilogue
        const uint32_t bw = ((uint32_t)S.y << A.h) | (uint32_t)li.x;
        double part = 0.0;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if (off[m] < 0) continue;
            const int i = p + m * per_pass;
            const int rb = i * Lp + j;
            double dn = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) dn += xt[rb + lof[q]];
            const int32_t *ul = A.ulo + (U.z + i) * 9;
            const int nu = ul[0];
            for (int q = 0; q < nu; ++q) dn += xt[rb + ul[1 + q] * Lp];
            const uint32_t aw = A.lwords[U.x + i];
            const double dg = A.u0 * (double)__popc(aw & bw);
            double y = ef.x * (A.hop * (acc[m] + dn) + dg * x0[m]);
            if (A.z) y -= ef.y * A.z[off[m]];
            A.y[off[m]] = y;
            part += x0[m] * y;
        }
        if (A.partials) {
            const double sum = block_sum(part, red);
            if (tid == 0) A.partials[it.slot] = sum;
        }
    }
}

hipError_t launch_hubseg(const ecut_sectors *s, const HubSegArgs &args, int grid, int n_xcd, hipStream_t st) {
    HubSegArgs A = args;
    if (n_xcd != 1) n_xcd = 8;
    if (grid % n_xcd) grid = (grid / n_xcd) * n_xcd;
    if (grid < n_xcd) grid = n_xcd;
    A.n_xcd = n_xcd;
    A.per_xcd = (A.n_items + n_xcd - 1) / n_xcd;
    const size_t lds = (size_t)s->hs_max_tile * 8;
    hipLaunchKernelGGL(k_hubseg, dim3(grid), dim3(HUBSEG_THREADS), lds, st, A);
    return hipGetLastError();
}

size_t hub3_lds_bytes(const ecut_sectors *s) {
    auto al = [](size_t b) { return (b + 15) & ~(size_t)15; };
    const int mns = s->hub.max_nseg;
    return al((size_t)s->h3_max_tile * 8) + al((size_t)mns * 16) + al((size_t)mns * s->h3_hs * 4) + al((size_t)mns * 4) +
           (size_t)s->h3.max_l * 48;
}

hipError_t launch_hub3(const ecut_sectors *s, const Hub3Args &args, int grid, int n_xcd, bool split, int slab_grid,
                       hipStream_t st) {
    Hub3Args A = args;
    if (grid % n_xcd) grid = (grid / n_xcd) * n_xcd;
    if (grid < n_xcd) grid = n_xcd;
    A.n_xcd = n_xcd;
    A.per_xcd = (A.n_items + n_xcd - 1) / n_xcd;
    if (split && slab_grid > 0) {
        // pass 1: left operator over column slabs held in L2; pass 2: tiles
        hipLaunchKernelGGL(k_upslab, dim3(slab_grid), dim3(SLAB_THREADS), 0, st, A.x, A.y, A.hl_ptr, A.hl_col, A.hl_val,
                           A.n_rows, A.dR, slab_grid / 8);
    }
    const bool stream = (int64_t)A.n_rows * A.dR >= STREAM_STORE_MIN;
    const size_t lds = hub3_lds_bytes(s);
    if (split && stream)
        hipLaunchKernelGGL((k_hub3<false, true>), dim3(grid), dim3(HUB3_THREADS), lds, st, A);
    else if (split)
        hipLaunchKernelGGL((k_hub3<false, false>), dim3(grid), dim3(HUB3_THREADS), lds, st, A);
    else if (stream)
        hipLaunchKernelGGL((k_hub3<true, true>), dim3(grid), dim3(HUB3_THREADS), lds, st, A);
    else
        hipLaunchKernelGGL((k_hub3<true, false>), dim3(grid), dim3(HUB3_THREADS), lds, st, A);
    return hipGetLastError();
}

int hub_blocks_per_cu(int which, size_t lds) {
    int n = 0;
    hipError_t e = hipSuccess;
    if (which == 3) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)k_hub3<true, true>, HUB3_THREADS, lds);
    else if (which == 4) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)k_upslab, SLAB_THREADS, 0);
    else if (which == 5) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)k_hubseg, HUBSEG_THREADS, lds);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void *)k_hub2<true, true>, HUB2_THREADS, lds);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    return n > 0 ? n : 1;
}

size_t hub2_lds_bytes(const ecut_sectors *s) {
    const HubDev &H = s->hub;
    const int nlo = 1 << H.h, nhi = 1 << (H.n_r - H.h);
    auto al = [](size_t b) { return (b + 15) & ~(size_t)15; };
    size_t b = al((size_t)H.max_tile * 8) + 3 * al((size_t)H.max_nseg * 4) + al((size_t)H.max_nseg * H.cls_hi_stride * 4);
    b += al((size_t)nhi * 4) + al((size_t)nlo * 4) + al((size_t)(H.n_coef > 0 ? H.n_coef : 1) * 8);
    return b;
}

hipError_t launch_hub2(const ecut_sectors *s, const ProblemDev &prob, const HubItem *items_d, int n_items, int grid,
                       int n_xcd, hipStream_t st) {
    const size_t lds = hub2_lds_bytes(s);
    if (grid % n_xcd) grid = (grid / n_xcd) * n_xcd;
    if (grid < n_xcd) grid = n_xcd;
    const int per_xcd = (n_items + n_xcd - 1) / n_xcd;
    const HubDev &H = s->hub;
    if (H.uniform_u && H.uniform_t)
        hipLaunchKernelGGL((k_hub2<true, true>), dim3(grid), dim3(HUB2_THREADS), lds, st, prob, items_d, n_items, n_xcd,
                           per_xcd);
    else
        hipLaunchKernelGGL((k_hub2<false, false>), dim3(grid), dim3(HUB2_THREADS), lds, st, prob, items_d, n_items,
                           n_xcd, per_xcd);
    return hipGetLastError();
}

size_t hub_lds_bytes(const ecut_sectors *s) {
    const HubDev &H = s->hub;
    const int dR = s->blocks[0].d_r;
    const int nlo = 1 << H.h, nhi = 1 << (H.n_r - H.h);
    auto al = [](size_t b) { return (b + 15) & ~(size_t)15; };
    size_t b = al((size_t)dR * 8) + al((size_t)dR * (H.n_r <= 16 ? 2 : 4));
    b += al((size_t)nlo * 4) * 2 + al((size_t)nlo * H.lo_stride * 4);
    b += al((size_t)nhi * 4) * 2 + al((size_t)nhi * H.hi_stride * 4);
    b += al((size_t)(H.n_coef > 0 ? H.n_coef : 1) * 8);
    if (!H.uniform_u) b += 3 * 256 * 8;
    return b;
}

// ------------------------------------------------------------------------
// Two-pass Hubbard application on flat work items (any hopping graph).
//
// The left operator H_up (x) 1 combines whole rows: every row is read by its
// ~8 neighbours, which must find it in L2 for the gather not to cost one HBM
// (or last-level-cache) read per neighbour.  The right operator 1 (x) H_dn
// gathers inside a row, whose class of columns is too wide to keep the left
// operator's neighbour window on chip at the same time.  So the two operators
// run as two passes over the vector:
//   pass 1 (k_hubU): y = H_up x on column slabs, items slab-major with the
//           rows of a slab in level order, so the blocks an XCD has in flight
//           share their neighbour rows;
//   pass 2 (k_hubD): y = xscale (y + H_dn x + D x) - zcoef z on runs of whole
//           rows, the in-row gathers served from L2, plus one partial
//           <x, y> per item for the Lanczos step.
// Both launches are one block per item (no persistent loop): the hardware
// dispatches blocks in index order, so an XCD's blocks in flight are always a
// contiguous window of its item range.  Block b runs on XCD b % 8 and takes
// item (b % 8) * per_xcd + b / 8 (n_xcd == 8), or item b (n_xcd == 1).
// ------------------------------------------------------------------------
__device__ __forceinline__ int xcd_item(int n_xcd, int per_xcd) {
    return n_xcd == 8 ? (int)(blockIdx.x & 7u) * per_xcd + (int)(blockIdx.x >> 3) : (int)blockIdx.x;
}

// A wave takes every (4 / ways)-th row of its item (at most HUBU_RMAX).  Its
// rows' CSR ranges, output rows and source rows are loaded once, one entry
// per lane, and read back with readlane, so the gathers of a row wait for no
// index load of their own.
template <bool PAIR, bool STREAM, bool OFF32>
__device__ __forceinline__ void hubU_item(const HubUArgs &A, int it) {
    const int sg = it / A.n_rgroups;
    const int rg = it - sg * A.n_rgroups;
    constexpr int CPL = PAIR ? 2 : 1;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // wave w takes slab w % ways of the group and every (4 / ways)-th row
    const int ways = A.slab_ways;
    const int slab = sg * ways + wave % ways;
    const int c = (slab * 64 + lane) * CPL;
    const bool ok = c < A.dR;
    // lanes past the row end gather column 0 (always present) instead of
    // masking every load; their store is the one thing skipped
    const int cl = ok ? c : 0;
    const int64_t dR = A.dR;
    const int step = HUBU_THREADS / 64 / ways;
    const int r0 = rg * A.rows_per_item + wave / ways;
    const int r1 = min(rg * A.rows_per_item + A.rows_per_item, A.n_rows);
    const int nrw = r0 < r1 ? min((r1 - r0 + step - 1) / step, HUBU_RMAX) : 0;
    int pa = 0, pb = 0, ar = 0;
    if (lane < nrw) {
        const int rr = r0 + lane * step;
        pa = A.hl_ptr[rr];
        pb = A.hl_ptr[rr + 1];
        ar = A.rows[rr];
    }
    // OFF32 (the vector's bytes fit 32 bits): the neighbour rows' byte
    // offsets, added to the lane's own, so a gather is one 32-bit add
    // beside the scalar base instead of a 64-bit row product per neighbour
    int colv[HUBU_RMAX];
    const uint32_t row_bytes = 8u * (uint32_t)A.dR;
#pragma unroll
    for (int k = 0; k < HUBU_RMAX; ++k) {
        colv[k] = 0;
        if (k < nrw) {
            const int q0 = __builtin_amdgcn_readlane(pa, k);
            if (lane < __builtin_amdgcn_readlane(pb, k) - q0) {
                const int col = A.hl_col[q0 + lane];
                colv[k] = OFF32 ? (int)((uint32_t)col * row_bytes) : col;
            }
        }
    }
    const double *__restrict__ xc = A.x + cl;
    const uint32_t lane_bytes = 8u * (uint32_t)cl;
    auto nb_src = [&](int k, int n) -> const double * {
        const int v = __builtin_amdgcn_readlane(colv[k], n);
        if constexpr (OFF32) return (const double *)((const char *)A.x + ((uint32_t)v + lane_bytes));
        else return xc + (int64_t)v * dR;
    };
#pragma unroll
    for (int k = 0; k < HUBU_RMAX; ++k) {
        if (k >= nrw) break;
        const int q0 = __builtin_amdgcn_readlane(pa, k);
        const int deg = __builtin_amdgcn_readlane(pb, k) - q0;
        const int a = __builtin_amdgcn_readlane(ar, k);
        const double *__restrict__ hv = A.hl_val + q0;
        double acc0 = 0.0, acc1 = 0.0;
        int j = 0;
        // whole batches: every load of a batch is issued before any is
        // consumed, with no per-neighbour test
        for (; j + HUBU_NB <= deg; j += HUBU_NB) {
            double v0[HUBU_NB], v1[HUBU_NB], h[HUBU_NB];
#pragma unroll
            for (int u = 0; u < HUBU_NB; ++u) {
                const double *p = nb_src(k, j + u);
                if constexpr (PAIR) {
                    const double2 q = *(const double2 *)p;
                    v0[u] = q.x;
                    v1[u] = q.y;
                } else {
                    v0[u] = *p;
                    v1[u] = 0.0;
                }
            }
            if (!A.uniform) {
#pragma unroll
                for (int u = 0; u < HUBU_NB; ++u) h[u] = hv[j + u];
            }
#pragma unroll
            for (int u = 0; u < HUBU_NB; ++u) {
                const double hu = A.uniform ? 1.0 : h[u];
                acc0 += hu * v0[u];
                acc1 += hu * v1[u];
            }
        }
        // the last, partial batch (same order of terms)
        if (j < deg) {
            double v0[HUBU_NB], v1[HUBU_NB];
#pragma unroll
            for (int u = 0; u < HUBU_NB; ++u) {
                v0[u] = v1[u] = 0.0;
                if (j + u < deg) {
                    const double *p = nb_src(k, j + u);
                    if constexpr (PAIR) {
                        const double2 q = *(const double2 *)p;
                        v0[u] = q.x;
                        v1[u] = q.y;
                    } else {
                        v0[u] = *p;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < HUBU_NB; ++u)
                if (j + u < deg) {
                    const double hu = A.uniform ? 1.0 : hv[j + u];
                    acc0 += hu * v0[u];
                    acc1 += hu * v1[u];
                }
        }
        if (A.uniform) {   // sum, then scale once
            acc0 *= A.hop;
            acc1 *= A.hop;
        }
        if (ok) {
            double *dst = A.y + (int64_t)a * dR + c;
            if constexpr (PAIR) {
                if constexpr (STREAM) {
                    __builtin_nontemporal_store(acc0, dst);
                    __builtin_nontemporal_store(acc1, dst + 1);
                } else {
                    *(double2 *)dst = make_double2(acc0, acc1);
                }
            } else {
                store_result<STREAM>(dst, acc0);
            }
        }
    }
}

template <bool PAIR, bool STREAM, bool OFF32>
__global__ __launch_bounds__(HUBU_THREADS) void k_hubU(const HubUArgs A, int n_xcd, int per_xcd) {
    const int it = xcd_item(n_xcd, per_xcd);
    if (it >= A.n_items) return;
    hubU_item<PAIR, STREAM, OFF32>(A, it);
}

// every byte offset into a vector of n elements (a 16-byte read at most)
// fits 32 bits
static bool fits_off32(int64_t n) { return n * 8 + 16 <= (int64_t)UINT32_MAX; }

// NS: bond slots held in registers (>= A.n_slots).  The source column of
// each bond for this thread's column is loaded once per item and reused for
// every row of it; a slot of -1 (the bond cannot hop from this column) reads
// nothing.  The terms of an amplitude are summed in slot order.
template <int NS, bool UNIF, bool STREAM>
__device__ __forceinline__ void hubD_item(const HubDArgs &A, int it, double *red) {
    const double2 ef = epi_factors(A.dscale, A.xscale, A.zcoef);
    const int rg = it / A.n_chunks;
    const int chunk = it - rg * A.n_chunks;
    const int c = chunk * HUBD_THREADS + (int)threadIdx.x;
    const bool ok = c < A.dR;
    const int64_t dR = A.dR;
    int src[NS];
    double hv[UNIF ? 1 : NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        src[k] = (ok && k < A.n_slots) ? A.col[(int64_t)k * dR + c] : -1;
        if constexpr (!UNIF) hv[k] = src[k] >= 0 ? A.val[(int64_t)k * dR + c] : 0.0;
    }
    const uint32_t bw = ok ? A.rwords[c] : 0u;
    const int r0 = rg * A.rows_per_item;
    const int r1 = min(r0 + A.rows_per_item, A.n_rows);
    double part = 0.0;
    if (ok) {
        for (int a = r0; a < r1; ++a) {
            const int64_t base = (int64_t)a * dR;
            const double *__restrict__ xr = A.x + base;
            const double x0 = xr[c];
            const double t = STREAM ? __builtin_nontemporal_load(A.y + base + c) : A.y[base + c];
            const double zv = A.z ? (STREAM ? __builtin_nontemporal_load(A.z + base + c) : A.z[base + c]) : 0.0;
            double dn = 0.0;
#pragma unroll
            for (int k0 = 0; k0 < NS; k0 += HUBD_NB) {
                double v[HUBD_NB];
#pragma unroll
                for (int k = 0; k < HUBD_NB; ++k) v[k] = src[k0 + k] >= 0 ? xr[src[k0 + k]] : 0.0;
#pragma unroll
                for (int k = 0; k < HUBD_NB; ++k) dn += UNIF ? v[k] : hv[k0 + k] * v[k];
            }
            const uint32_t both = A.lwords[a] & bw;
            double dg;
            if (A.uniform_u) {
                dg = A.u0 * (double)__popc(both);
            } else {
                dg = 0.0;
                for (uint32_t m = both; m; m &= m - 1u) dg += A.u[__ffs(m) - 1];
            }
            double y = UNIF ? ef.x * (t + A.hop * dn + dg * x0) : ef.x * (t + dn + dg * x0);
            if (A.z) y -= ef.y * zv;
            store_result<STREAM>(A.y + base + c, y);
            part += x0 * y;
        }
    }
    if (A.partials) {
        const double sum = block_sum(part, red);
        if (threadIdx.x == 0) A.partials[it] = sum;
    }
}

template <int NS, bool UNIF, bool STREAM>
__global__ __launch_bounds__(HUBD_THREADS) void k_hubD(const HubDArgs A, int n_xcd, int per_xcd) {
    __shared__ double red[HUBD_THREADS / 64];
    const int it = xcd_item(n_xcd, per_xcd);
    if (it >= A.n_items) return;   // uniform over the block
    hubD_item<NS, UNIF, STREAM>(A, it, red);
}

// Problem of global item `it` of a batch: the last p with off[p] <= it.
__device__ __forceinline__ int batch_problem(const int32_t *__restrict__ off, int n_probs, int it) {
    int lo = 0, hi = n_probs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= it) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Batches of Hubbard problems: one launch per pass over the items of every
// problem (problem p owns items off[p] .. off[p + 1] - 1, its own item
// numbering inside), each item computed exactly as in its problem's own
// launch.  Column pairs, hop values and the slot count are per problem.
__global__ __launch_bounds__(HUBU_THREADS) void k_hubU_batch(const HubUArgs *__restrict__ probs,
                                                             const int32_t *__restrict__ off, int n_probs,
                                                             int n_items, int per_xcd) {
    const int it = xcd_item(8, per_xcd);
    if (it >= n_items) return;
    const int p = batch_problem(off, n_probs, it);
    const HubUArgs A = probs[p];
    const bool pair = (A.dR % 2 == 0) && !(((uintptr_t)A.x | (uintptr_t)A.y) & 15);
    if (pair) hubU_item<true, false>(A, it - off[p]);
    else hubU_item<false, false>(A, it - off[p]);
}

__global__ __launch_bounds__(HUBD_THREADS) void k_hubD_batch(const HubDArgs *__restrict__ probs,
                                                             const int32_t *__restrict__ off, int n_probs,
                                                             int n_items, int per_xcd) {
    __shared__ double red[HUBD_THREADS / 64];
    const int it = xcd_item(8, per_xcd);
    if (it >= n_items) return;
    const int p = batch_problem(off, n_probs, it);
    const HubDArgs A = probs[p];
    if (A.val == nullptr) hubD_item<HUBD_BATCH_SLOTS, true, false>(A, it - off[p], red);
    else hubD_item<HUBD_BATCH_SLOTS, false, false>(A, it - off[p], red);
}

hipError_t launch_hub6_batch(const HubUArgs *probs_u, const HubDArgs *probs_d, const int32_t *off_u,
                             const int32_t *off_d, int n_probs, int n_items_u, int n_items_d, hipStream_t st) {
    if (n_probs <= 0) return hipSuccess;
    const int pu = (n_items_u + 7) / 8, pd = (n_items_d + 7) / 8;
    hipLaunchKernelGGL(k_hubU_batch, dim3(8 * pu), dim3(HUBU_THREADS), 0, st, probs_u, off_u, n_probs, n_items_u, pu);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hubD_batch, dim3(8 * pd), dim3(HUBD_THREADS), 0, st, probs_d, off_d, n_probs, n_items_d, pd);
    return hipGetLastError();
}

template <int NS>
static void launch_hubD(const HubDArgs &D, bool stream, dim3 grid, int xu, int pd, hipStream_t st) {
    const bool unif = D.val == nullptr;
    if (unif && stream) hipLaunchKernelGGL((k_hubD<NS, true, true>), grid, dim3(HUBD_THREADS), 0, st, D, xu, pd);
    else if (unif) hipLaunchKernelGGL((k_hubD<NS, true, false>), grid, dim3(HUBD_THREADS), 0, st, D, xu, pd);
    else if (stream) hipLaunchKernelGGL((k_hubD<NS, false, true>), grid, dim3(HUBD_THREADS), 0, st, D, xu, pd);
    else hipLaunchKernelGGL((k_hubD<NS, false, false>), grid, dim3(HUBD_THREADS), 0, st, D, xu, pd);
}

hipError_t launch_hub6_left(const HubUArgs &U, int n_xcd, hipStream_t st) {
    const bool pair = (U.dR % 2 == 0) && !(((uintptr_t)U.x | (uintptr_t)U.y) & 15);
    const bool stream = (int64_t)U.n_rows * U.dR >= STREAM_STORE_MIN;
    const int xu = n_xcd == 1 ? 1 : 8;
    const int pu = (U.n_items + xu - 1) / xu;
    const dim3 gu(xu == 8 ? 8 * pu : U.n_items);
    const bool o32 = fits_off32((int64_t)U.n_rows * U.dR);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, gu, dim3(HUBU_THREADS), 0, st, U, xu, pu); };
    if (o32) {
        if (pair && stream) go(k_hubU<true, true, true>);
        else if (pair) go(k_hubU<true, false, true>);
        else if (stream) go(k_hubU<false, true, true>);
        else go(k_hubU<false, false, true>);
    } else {
        if (pair && stream) go(k_hubU<true, true, false>);
        else if (pair) go(k_hubU<true, false, false>);
        else if (stream) go(k_hubU<false, true, false>);
        else go(k_hubU<false, false, false>);
    }
    return hipGetLastError();
}

hipError_t launch_hubD_only(const HubDArgs &D, int n_xcd, hipStream_t st) {
    const bool stream = (int64_t)D.n_rows * D.dR >= STREAM_STORE_MIN;
    const int xu = n_xcd == 1 ? 1 : 8;
    const int pd = (D.n_items + xu - 1) / xu;
    const dim3 gd(xu == 8 ? 8 * pd : D.n_items);
    if (D.n_slots <= 8) launch_hubD<8>(D, stream, gd, xu, pd, st);
    else if (D.n_slots <= 16) launch_hubD<16>(D, stream, gd, xu, pd, st);
    else if (D.n_slots <= HUBD_MAX_SLOTS) launch_hubD<HUBD_MAX_SLOTS>(D, stream, gd, xu, pd, st);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// c+ / c of one mode between Hubbard up/down sectors (Krylov dynamical
// correlations).  Fermion order: up modes, then down modes, each by site;
// the sign is (-1)^(occupied modes before the mode) in the source word: the
// up particles below the site for an up mode, every up particle plus the
// down particles below the site for a down mode.  The destination word
// has the mode occupied for c+ and empty for c; the source word is the
// destination word with the mode flipped, found by its colex rank.
// ------------------------------------------------------------------------
__device__ __forceinline__ int64_t colex_rank_dev(uint32_t w, const uint64_t *__restrict__ binom) {
    int64_t r = 0;
    int j = 0;
    while (w) {
        const int p = __ffs(w) - 1;
        r += (int64_t)binom[p * 65 + j + 1];
        ++j;
        w &= w - 1u;
    }
    return r;
}

__global__ __launch_bounds__(256) void k_cdag(const CdagArgs A) {
    const uint32_t bit = 1u << A.site;
    const uint32_t below = bit - 1u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.dim; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = i / A.dR_dst;
        const int c = (int)(i - a * A.dR_dst);
        const uint32_t uw = A.dst_lwords[a];
        const uint32_t dw = A.dst_rwords[c];
        const uint32_t mw = A.spin == 0 ? uw : dw;
        double v = 0.0;
        if (((mw & bit) != 0) == (A.dagger != 0)) {
            const uint32_t sw = mw ^ bit;   // the source word of the mode's spin
            int par;
            int64_t src;
            if (A.spin == 0) {
                par = __popc(sw & below);
                src = colex_rank_dev(sw, A.binom) * A.dR_src + c;
            } else {
                par = __popc(uw) + __popc(sw & below);
                const int64_t r = colex_rank_dev(sw, A.binom);
                src = a * A.dR_src + (A.src_col_of_rank ? A.src_col_of_rank[r] : r);
            }
            const double xv = A.x[src];
            v = (par & 1) ? -xv : xv;
        }
        A.y[i] = v;
    }
}

// colex unrank: the idx-th word with k set bits
__device__ __forceinline__ uint32_t colex_unrank_dev(int64_t idx, int k, const uint64_t *__restrict__ binom) {
    uint32_t w = 0;
    for (int j = k; j >= 1; --j) {
        int p = j - 1;
        while ((int64_t)binom[(p + 1) * 65 + j] <= idx) ++p;
        w |= 1u << p;
        idx -= (int64_t)binom[p * 65 + j];
    }
    return w;
}

// bits of w at the set positions of mask, packed to the low bits in order
__device__ __forceinline__ uint32_t compact_dev(uint32_t w, uint32_t mask) {
    uint32_t out = 0;
    int k = 0;
    for (uint32_t m = mask; m; m &= m - 1u, ++k) out |= ((w >> (__ffs(m) - 1)) & 1u) << k;
    return out;
}

// canonical <-> bipartite layout of the spatial Hubbard cut (see
// build_hubbard_spatial): position of the canonical index and the parity of
// reordering its modes from (all up, all down) to (L up, L down, R up,
// R down): every R up particle below an L up particle, every R down particle
// below an L down particle, and every (R up, L down) pair.
__global__ __launch_bounds__(256) void k_perm_hubsp(const HubSpPerm A, const double *__restrict__ in,
                                                    double *__restrict__ out, int to_bip) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.dim; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t iu = i / A.n_dn_words, id = i - iu * A.n_dn_words;
        const uint32_t up = colex_unrank_dev(iu, A.n_up, A.binom), dn = colex_unrank_dev(id, A.n_dn, A.binom);
        const uint32_t ul = compact_dev(up, A.lmask), dl = compact_dev(dn, A.lmask);
        const uint32_t ur = compact_dev(up, A.rmask), dr = compact_dev(dn, A.rmask);
        const int a = __popc(ul), b = __popc(dl);
        const int q = (a - A.la0) * A.nb_b + (b - A.lb0);
        const BlockDev B = A.blocks[q];
        const int64_t row = colex_rank_dev(ul, A.binom) * (int64_t)A.binom[A.nL * 65 + b] + colex_rank_dev(dl, A.binom);
        const int64_t col = colex_rank_dev(ur, A.binom) * (int64_t)A.binom[A.nR * 65 + (A.n_dn - b)] +
                            colex_rank_dev(dr, A.binom);
        const int64_t pos = B.offset + row * B.d_r + col;
        int par = __popc(ur) * b;
        for (uint32_t m = A.lmask; m; m &= m - 1u) {
            const uint32_t below = (m & (0u - m)) - 1u;   // sites below this L site
            const int site_bit = __ffs(m) - 1;
            if ((up >> site_bit) & 1u) par += __popc(up & A.rmask & below);
            if ((dn >> site_bit) & 1u) par += __popc(dn & A.rmask & below);
        }
        if (to_bip) {
            const double v = in[i];
            out[pos] = (par & 1) ? -v : v;
        } else {
            const double v = in[pos];
            out[i] = (par & 1) ? -v : v;
        }
    }
}

hipError_t launch_perm_hubsp(const HubSpPerm &A, const double *in, double *out, bool to_bip, hipStream_t st) {
    if (A.dim == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((A.dim + 255) / 256, 65536);
    hipLaunchKernelGGL(k_perm_hubsp, dim3((unsigned)blocks), dim3(256), 0, st, A, in, out, to_bip ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_cdag(const CdagArgs &A, hipStream_t st) {
    const int64_t blocks = std::min<int64_t>((A.dim + 255) / 256, 65536);
    hipLaunchKernelGGL(k_cdag, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, A);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// canonical <-> bipartite permutations (spin spatial cut).  The canonical
// index is unranked into the full word, split by the cut mask, and the two
// halves ranked again.
// ------------------------------------------------------------------------
struct PermDev {
    const uint64_t *binom;    // [65][65]
    const BlockDev *blocks;
    uint64_t left_mask;
    int32_t n_sites, n_up, qmin, pad;
};

__device__ __forceinline__ uint64_t dbinom(const uint64_t *bt, int n, int k) {
    return (k < 0 || k > n) ? 0ull : bt[n * 65 + k];
}

__device__ int64_t d_canon_to_pos(const PermDev &D, int64_t idx) {
    // unrank the canonical index into the full word (colex)
    uint64_t w = 0;
    int p = D.n_sites - 1;
    for (int j = D.n_up; j >= 1; --j) {
        while (p >= j && (int64_t)dbinom(D.binom, p, j) > idx) --p;
        w |= 1ull << p;
        idx -= (int64_t)dbinom(D.binom, p, j);
        --p;
    }
    // split and rank both halves
    int64_t rl = 0, rr = 0;
    int kl = 0, kr = 0, bl = 0, br = 0;
    for (int s = 0; s < D.n_sites; ++s) {
        const bool set = (w >> s) & 1ull;
        if ((D.left_mask >> s) & 1ull) {
            if (set) { ++kl; rl += (int64_t)dbinom(D.binom, bl, kl); }
            ++bl;
        } else {
            if (set) { ++kr; rr += (int64_t)dbinom(D.binom, br, kr); }
            ++br;
        }
    }
    const BlockDev B = D.blocks[kl - D.qmin];
    return B.offset + rl * B.d_r + rr;
}

__global__ void k_import(PermDev D, const double *__restrict__ canon, double *__restrict__ bip, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        bip[d_canon_to_pos(D, i)] = canon[i];
}

__global__ void k_export(PermDev D, const double *__restrict__ bip, double *__restrict__ canon, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        canon[i] = bip[d_canon_to_pos(D, i)];
}

// Hubbard block with permuted columns: canonical index i = a * dR + r (up
// rank a, down rank r) sits at a * dR + col[r].
__global__ void k_perm_cols(const int32_t *__restrict__ col, int64_t n_rows, int dR, const double *__restrict__ in,
                            double *__restrict__ out, int to_bip) {
    const int64_t n = n_rows * dR;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = i / dR;
        const int64_t p = a * dR + col[i - a * dR];
        if (to_bip) out[p] = in[i];
        else out[i] = in[p];
    }
}

hipError_t launch_perm_cols(const int32_t *col_d, int64_t n_rows, int dR, const double *in, double *out, bool to_bip,
                            hipStream_t st) {
    const int64_t n = n_rows * dR;
    int grid = (int)((n + 255) / 256);
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_perm_cols, dim3(grid), dim3(256), 0, st, col_d, n_rows, dR, in, out, to_bip ? 1 : 0);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// Lanczos vector kernels.  A "segment set" describes one vector per problem
// for batched launches: seg k covers [0, n_k) of vectors x_k, y_k.
// ------------------------------------------------------------------------
// Next-step factors of the Lanczos recurrence, done by the thread that
// finishes the |w|^2 reduction of a solve (VecJob::next): with
// beta = |w| the next vector is w / beta, so the next apply scales by 1/beta
// and subtracts beta s_j w_j.  A zero or non-finite beta makes the factors
// non-finite; the host sees the breakdown in the copied scalars and stops the
// solve.
__device__ __forceinline__ void lz_next(const LzNextJob &J) {
    double *s = J.scal;
    const double a = s[0], b2 = s[1];
    const double beta = sqrt(b2 > 0.0 ? b2 : 0.0);
    const double inv = 1.0 / beta;
    s[LZ_Z] = J.start ? 0.0 : beta * s[LZ_S];
    s[LZ_S] = inv;
    if (J.scales) J.scales[J.slot] = inv;
    J.out2[0] = a;
    J.out2[1] = b2;
}

__global__ __launch_bounds__(VEC_THREADS) void k_reduce(const VecJob *__restrict__ jobs, int n_jobs) {
    __shared__ double red[VEC_THREADS / 64];
    const int j = blockIdx.x;
    if (j >= n_jobs) return;
    const VecJob J = jobs[j];
    double s = 0.0;
    // fixed assignment of partial slots to threads, then a fixed-order block
    // sum; eight loads in flight, added in slot order
    const int nt = blockDim.x;
    int i = threadIdx.x;
    for (; i + 7 * nt < J.n_partials; i += 8 * nt) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = J.partials[i + k * nt];
#pragma unroll
        for (int k = 0; k < 8; ++k) s += v[k];
    }
    for (; i < J.n_partials; i += nt) s += J.partials[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        if (J.mode == 0) J.scalars[J.out] = (J.dscale ? J.dscale[0] : J.scale) * s;
        else J.scalars[J.out] = s;
        if (J.next.scal) lz_next(J.next);
    }
}

// y <- y - (scalars[coef_idx] * coef_mul) * x ; partials[chunk] = sum y^2
__global__ __launch_bounds__(VEC_THREADS) void k_axpy_norm(const VecJob *__restrict__ jobs, const int32_t *__restrict__ chunk_job,
                                                           const int32_t *__restrict__ chunk_idx, int n_chunks) {
    __shared__ double red[VEC_THREADS / 64];
    __shared__ double bcast;
    for (int c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const VecJob J = jobs[chunk_job[c]];
        const int ci = chunk_idx[c];
        const int64_t ck = J.chunk > 0 ? J.chunk : VEC_CHUNK;
        const int64_t i0 = (int64_t)ci * ck;
        const int64_t i1 = i0 + ck < J.n ? i0 + ck : J.n;
        double sc = J.dscale ? J.dscale[0] : J.coef_mul;
        double a;
        if (J.a_partials) {
            // the coefficient's reduction, done here in k_reduce's order so
            // every block (and the stored value) gets k_reduce's result
            double t = 0.0;
            for (int i = threadIdx.x; i < J.a_n; i += blockDim.x) t += J.a_partials[i];
            t = block_sum(t, red);   // the sum in thread 0, after a barrier
            if (threadIdx.x == 0) bcast = t;
            __syncthreads();
            t = bcast;               // read before the norm's block_sum barriers below
            const double coef = (J.dscale ? J.dscale[0] : J.scale) * t;
            if (ci == 0 && threadIdx.x == 0) J.scalars[J.coef_idx] = coef;
            a = coef * sc;
        } else {
            a = J.scalars[J.coef_idx] * sc;
        }
        // eight elements per thread and pass, all loads before any store;
        // each thread still takes i0 + tid, + blockDim, ... in order
        const double *__restrict__ xp = J.x;
        double *__restrict__ yp = J.y;
        double s = 0.0;
        for (int64_t base = i0 + threadIdx.x; base < i1; base += 8 * (int64_t)blockDim.x) {
            double yv[8], xv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t i = base + (int64_t)u * blockDim.x;
                yv[u] = i < i1 ? yp[i] : 0.0;
                xv[u] = i < i1 ? xp[i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t i = base + (int64_t)u * blockDim.x;
                if (i < i1) {
                    const double v = yv[u] - a * xv[u];
                    yp[i] = v;
                    s += v * v;
                }
            }
        }
        s = block_sum(s, red);
        if (threadIdx.x == 0) J.partials[ci] = s;
    }
}

// Reorthogonalisation kernels.  One work group per chunk of VEC_CHUNK
// elements (512 threads x 16 elements); a thread's chunk of y stays in
// registers while the basis vectors stream past it.  Element pair t of a
// thread is (i0 + 2 (tid + 512 t), i0 + 2 (tid + 512 t) + 1); with V2 (every
// vector 16-byte aligned, even ld) a pair is one 16-byte load.
constexpr int CGS_THREADS = 512;
constexpr int CGS_PAIRS = (int)(VEC_CHUNK / (2 * CGS_THREADS));
static_assert(2 * CGS_THREADS * CGS_PAIRS == VEC_CHUNK, "one chunk per work group");

template <bool V2>
__device__ __forceinline__ void cgs_load(const double *__restrict__ p, int64_t i0, int64_t i1, double2 (&v)[CGS_PAIRS]) {
#pragma unroll
    for (int t = 0; t < CGS_PAIRS; ++t) {
        const int64_t e = i0 + 2 * (int64_t)(threadIdx.x + CGS_THREADS * t);
        if (e + 1 < i1)
            v[t] = V2 ? *(const double2 *)(p + e) : make_double2(p[e], p[e + 1]);
        else
            v[t] = make_double2(e < i1 ? p[e] : 0.0, 0.0);
    }
}

// Classical Gram-Schmidt, dot phase: partials[k * n_chunks + chunk] = <w_k, y> over the chunk.
// gate (nullable): when it points to 0.0 the kernel does nothing (the
// conditional second pass of the reorthogonalisation).  The per-wave sums of
// eight vectors are reduced across the group together, behind one barrier.
template <bool V2>
__global__ __launch_bounds__(CGS_THREADS) void k_multidot(const double *__restrict__ basis, int64_t ld, int nvec,
                                                          const double *__restrict__ y, int64_t n,
                                                          double *__restrict__ partials, int n_chunks,
                                                          const double *__restrict__ gate) {
    if (gate && *gate == 0.0) return;
    constexpr int NW = CGS_THREADS / 64;
    __shared__ double red[2][8][NW];   // two buffers: a group writes one while the other is read
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const int64_t i0 = (int64_t)c * VEC_CHUNK;
        const int64_t i1 = i0 + VEC_CHUNK < n ? i0 + VEC_CHUNK : n;
        double2 yv[CGS_PAIRS];
        cgs_load<V2>(y, i0, i1, yv);
        int g = 0;
        for (int k0 = 0; k0 < nvec; k0 += 8, g ^= 1) {
            double s[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                s[q] = 0.0;
                if (k0 + q < nvec) {
                    double2 b[CGS_PAIRS];
                    cgs_load<V2>(basis + (int64_t)(k0 + q) * ld, i0, i1, b);
#pragma unroll
                    for (int t = 0; t < CGS_PAIRS; ++t) {
                        s[q] += b[t].x * yv[t].x;
                        s[q] += b[t].y * yv[t].y;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) s[q] = wave_sum(s[q]);
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < 8; ++q) red[g][q][wid] = s[q];
            }
            __syncthreads();
            if (threadIdx.x < 8 && k0 + (int)threadIdx.x < nvec) {
                double r = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) r += red[g][threadIdx.x][w];
                partials[(int64_t)(k0 + threadIdx.x) * n_chunks + c] = r;
            }
        }
        __syncthreads();   // red is written again by the next chunk
    }
}

// coef[k] = scale_k * sum_chunks partials[k][*]  (fixed order)
__global__ __launch_bounds__(VEC_THREADS) void k_multidot_reduce(const double *__restrict__ partials, int n_chunks,
                                                                 const double *__restrict__ scale, double *__restrict__ coef,
                                                                 const double *__restrict__ gate) {
    if (gate && *gate == 0.0) return;
    __shared__ double red[VEC_THREADS / 64];
    const int k = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < n_chunks; i += blockDim.x) s += partials[(int64_t)k * n_chunks + i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) coef[k] = s * scale[k];
}

// y <- y - sum_k coef[k] * scale_k * w_k (sign != 0), or y <- sum_k ... (sign
// == 0); optional norm partials of the result per chunk.  Each element sums
// its terms in order k = 0, 1, ...  Capped at four waves per SIMD (at most
// 128 registers): the uncapped build holds more loads in flight but runs one
// group per compute unit, and streams the basis about 25% slower.
template <bool V2>
__global__ __launch_bounds__(CGS_THREADS, 4) void k_multiaxpy(const double *__restrict__ basis, int64_t ld, int nvec,
                                                           const double *__restrict__ coef, const double *__restrict__ scale,
                                                           double *__restrict__ y, int64_t n, double *__restrict__ partials,
                                                           int n_chunks, double sign, const double *__restrict__ gate) {
    if (gate && *gate == 0.0) return;
    __shared__ double red[CGS_THREADS / 64];
    __shared__ double cs[MAX_BASIS];
    for (int k = threadIdx.x; k < nvec; k += blockDim.x) cs[k] = coef[k] * scale[k];
    __syncthreads();
    for (int c = blockIdx.x; c < n_chunks; c += gridDim.x) {
        const int64_t i0 = (int64_t)c * VEC_CHUNK;
        const int64_t i1 = i0 + VEC_CHUNK < n ? i0 + VEC_CHUNK : n;
        double2 v[CGS_PAIRS];
#pragma unroll
        for (int t = 0; t < CGS_PAIRS; ++t) v[t] = make_double2(0.0, 0.0);
        // eight vectors per unrolled group, as in the dot kernel, so that
        // loads of later vectors can go out early
        for (int k0 = 0; k0 < nvec; k0 += 8) {
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (k0 + q < nvec) {
                    double2 b[CGS_PAIRS];
                    cgs_load<V2>(basis + (int64_t)(k0 + q) * ld, i0, i1, b);
                    const double ck = cs[k0 + q];
#pragma unroll
                    for (int t = 0; t < CGS_PAIRS; ++t) {
                        v[t].x += ck * b[t].x;
                        v[t].y += ck * b[t].y;
                    }
                }
            }
        }
        double2 yo[CGS_PAIRS];
        if (sign != 0.0) cgs_load<V2>(y, i0, i1, yo);
        double s = 0.0;
#pragma unroll
        for (int t = 0; t < CGS_PAIRS; ++t) {
            const int64_t e = i0 + 2 * (int64_t)(threadIdx.x + CGS_THREADS * t);
            const double2 r = sign != 0.0 ? make_double2(yo[t].x - v[t].x, yo[t].y - v[t].y) : v[t];
            if (e + 1 < i1) {
                if (V2) {
                    *(double2 *)(y + e) = r;
                } else {
                    y[e] = r.x;
                    y[e + 1] = r.y;
                }
                s += r.x * r.x;
                s += r.y * r.y;
            } else if (e < i1) {
                y[e] = r.x;
                s += r.x * r.x;
            }
        }
        if (partials) {
            s = block_sum(s, red);
            if (threadIdx.x == 0) partials[c] = s;
        }
    }
}

// Second-pass test of the reorthogonalisation (Daniel, Gragg, Kaufman and
// Stewart, 1976): project again only when the first projection removed more
// than half of the squared norm, ||w'||^2 < ||w||^2 / 2.
// s[2] = ||w||^2 before, s[3] = ||w'||^2 after the first pass; s[4] = gate.
__global__ void k_dgks_gate(double *s) {
    if (threadIdx.x == 0 && blockIdx.x == 0) s[4] = (s[3] < 0.5 * s[2]) ? 1.0 : 0.0;
}

hipError_t launch_dgks_gate(double *scal, hipStream_t st) {
    hipLaunchKernelGGL(k_dgks_gate, dim3(1), dim3(64), 0, st, scal);
    return hipGetLastError();
}

// y <- a * x (a from scalars[idx] or host value when scalars == NULL)
__global__ void k_scale_copy(const double *__restrict__ x, double *__restrict__ y, int64_t n, double a) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i];
}

// Seeded N(0,1) vector: splitmix64 of (seed, index) -> two uniforms -> Box-Muller.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_fill_normal(double *__restrict__ y, int64_t n, uint64_t seed) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t a = splitmix64(seed ^ splitmix64(2 * (uint64_t)i));
        const uint64_t b = splitmix64(seed ^ splitmix64(2 * (uint64_t)i + 1));
        const double u1 = ((double)(a >> 11) + 1.0) * (1.0 / 9007199254740993.0);   // (0,1]
        const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);           // [0,1)
        y[i] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    }
}

// ------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------
hipError_t launch_rows(const ProblemDev *probs_d, const ProblemDev &single, const ItemDev *items_d, int n_items,
                       int max_tile_elems, hipStream_t st) {
    if (n_items <= 0) return hipSuccess;
    const bool stage = (size_t)max_tile_elems * 8 <= ROWS_MAX_LDS;
    int grid = n_items < 65536 ? n_items : 65536;
    if (stage) {
        const size_t lds = (size_t)max_tile_elems * 8;
        hipLaunchKernelGGL(k_rows<true>, dim3(grid), dim3(ROWS_THREADS), lds, st, probs_d, single, items_d, n_items);
    } else {
        hipLaunchKernelGGL(k_rows<false>, dim3(grid), dim3(ROWS_THREADS), 0, st, probs_d, single, items_d, n_items);
    }
    return hipGetLastError();
}

hipError_t launch_spin(const ProblemDev *probs_d, const ProblemDev &single, const ItemDev *items_d, int n_items,
                       int max_tile_elems, int max_src, int grid, hipStream_t st) {
    if (n_items <= 0) return hipSuccess;
    if (max_tile_elems > SPIN_TILE || max_src > SPIN_TILE) return hipErrorInvalidValue;
    if (grid <= 0) grid = 2048;
    if (grid > n_items) grid = n_items;   // groups walk the list with a stride of the grid
    // one-row items: the row and the cross-term source rows; then the items of
    // several short rows (their tiles are at most SPIN_MANY_TILE)
    // the row buffer (the one-pass kernel sums the folded diagonal in place)
    const int cap = std::max(std::max(max_tile_elems, max_src), 1);
    const size_t lds1 = (size_t)cap * 8;
    hipLaunchKernelGGL(k_spin<true>, dim3(grid), dim3(SPIN_THREADS), lds1, st, probs_d, single, items_d, n_items, cap);
    const size_t lds2 = (size_t)SPIN_MANY_TILE * 8;
    hipLaunchKernelGGL(k_spin<false>, dim3(grid), dim3(SPIN_MANY_THREADS), lds2, st, probs_d, single, items_d, n_items,
                       0);
    return hipGetLastError();
}

hipError_t launch_spin2(const SpinLArgs &L, const ProblemDev &P, const uint16_t *tab, const int64_t *tbase,
                        const ItemDev *items_d, int n_one, int n_items, int max_d_r, int n_xcd, bool fermion,
                        hipStream_t st) {
    if (max_d_r > SPIN_TILE) return hipErrorInvalidValue;
    const int xu = n_xcd == 1 ? 1 : 8;
    auto grid_of = [&](int n, int &per) {
        per = (n + xu - 1) / xu;
        return dim3(xu == 8 ? 8 * per : n);
    };
    int per = 0;
    if (L.n_items > 0) {
        const dim3 g = grid_of(L.n_items, per);
        // 64-bit row products here: the 32-bit form of the Hubbard left pass
        // (fewer registers, eight waves per SIMD) measured slower on spin blocks
        if ((int64_t)P.dim >= STREAM_STORE_MIN)
            hipLaunchKernelGGL(k_spinL<true>, g, dim3(HUBU_THREADS), 0, st, L, xu, per);
        else
            hipLaunchKernelGGL(k_spinL<false>, g, dim3(HUBU_THREADS), 0, st, L, xu, per);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_one > 0) {
        const dim3 g = grid_of(n_one, per);
        const int cap = std::max(max_d_r, 1) + 1;   // + the zero slot
        const size_t lds = (size_t)(cap + XTAB_SLOTS) * 8;   // then the folded diagonal table
        const bool short_rows = max_d_r <= SPIN_SHORT_THREADS * SPIN_SHORT_M;
#define ECUT_SPINR(NT_, M_, F_)                                                                              \
    hipLaunchKernelGGL((k_spinR<true, NT_, M_, F_>), g, dim3(NT_), lds, st, P, tab, tbase, items_d, n_one, xu, per, cap)
        if (short_rows && fermion) ECUT_SPINR(SPIN_SHORT_THREADS, SPIN_SHORT_M, true);
        else if (short_rows) ECUT_SPINR(SPIN_SHORT_THREADS, SPIN_SHORT_M, false);
        else if (fermion) ECUT_SPINR(SPIN_THREADS, SPIN_M, true);
        else ECUT_SPINR(SPIN_THREADS, SPIN_M, false);
#undef ECUT_SPINR
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (n_items > n_one) {
        const dim3 g = grid_of(n_items - n_one, per);
        if (fermion) return hipErrorInvalidValue;   // the several-row items rank without signs
        hipLaunchKernelGGL((k_spinR<false, SPIN_THREADS, SPIN_M, false>), g, dim3(SPIN_MANY_THREADS),
                           (size_t)SPIN_MANY_TILE * 8, st, P, tab, tbase, items_d + n_one, n_items - n_one, xu, per, 0);
    }
    return hipGetLastError();
}

hipError_t launch_hub(const ecut_sectors *s, const ProblemDev &prob, const int32_t *rows_d, int n_rows, int grid,
                      int n_xcd, hipStream_t st) {
    const size_t lds = hub_lds_bytes(s);
    if (grid % n_xcd) grid = (grid / n_xcd) * n_xcd;
    if (grid < n_xcd) grid = n_xcd;
    const int per_xcd = (n_rows + n_xcd - 1) / n_xcd;
    const HubDev &H = s->hub;
    const bool w16 = H.n_r <= 16;
#define ECUT_HUB_LAUNCH(UU, UT, W)                                                                        \
    hipLaunchKernelGGL((k_hub<UU, UT, W>), dim3(grid), dim3(HUB_THREADS), lds, st, prob, rows_d, n_rows,  \
                       n_xcd, per_xcd)
    if (H.uniform_u && H.uniform_t && w16) ECUT_HUB_LAUNCH(true, true, true);
    else if (H.uniform_u && H.uniform_t) ECUT_HUB_LAUNCH(true, true, false);
    else if (w16) ECUT_HUB_LAUNCH(false, false, true);
    else ECUT_HUB_LAUNCH(false, false, false);
#undef ECUT_HUB_LAUNCH
    return hipGetLastError();
}

hipError_t set_hub_lds_limits(size_t bytes) {
    hipError_t e = hipSuccess;
    const int b = (int)bytes;
    e = hipFuncSetAttribute((const void *)k_spin<true>, hipFuncAttributeMaxDynamicSharedMemorySize, SPIN_TILE * 8);
    if (e != hipSuccess) return e;

    e = hipFuncSetAttribute((const void *)k_hubrow<1024, HUBROW_P, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            2 * HUBROW_P * 1024 * 10);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_hubrow<512, HUBROW_P, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            2 * HUBROW_P * 512 * 10);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_hubrow<512, HUBROW_P_SHORT, 4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            2 * HUBROW_P_SHORT * 512 * 10);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_hubrow<256, HUBROW_P, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            2 * HUBROW_P * 256 * 10);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_hub<true, true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_hub<true, true, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_hub<false, false, true>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_hub<false, false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_hub2<true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_hub2<false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_hub3<true, true>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_hub3<true, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_hub3<false, true>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_hub3<false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, b);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)k_rows<true>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ROWS_MAX_LDS);
}

hipError_t launch_perm(const ecut_sectors *s, const uint64_t *binom_d, const BlockDev *blocks_d, const double *in,
                       double *out, bool to_bip, hipStream_t st) {
    PermDev D{};
    D.binom = binom_d;
    D.blocks = blocks_d;
    D.left_mask = s->left_mask;
    D.n_sites = s->n_sites;
    D.n_up = s->n_up;
    D.qmin = s->blocks[0].q_l;
    const int64_t n = s->dim;
    int grid = (int)((n + 255) / 256);
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    if (to_bip) hipLaunchKernelGGL(k_import, dim3(grid), dim3(256), 0, st, D, in, out, n);
    else hipLaunchKernelGGL(k_export, dim3(grid), dim3(256), 0, st, D, in, out, n);
    return hipGetLastError();
}

hipError_t launch_reduce(const VecJob *jobs_d, int n_jobs, hipStream_t st) {
    if (n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(n_jobs), dim3(VEC_THREADS), 0, st, jobs_d, n_jobs);
    return hipGetLastError();
}

hipError_t launch_axpy_norm(const VecJob *jobs_d, const int32_t *chunk_job_d, const int32_t *chunk_idx_d, int n_chunks,
                            hipStream_t st) {
    if (n_chunks <= 0) return hipSuccess;
    int grid = n_chunks < 8192 ? n_chunks : 8192;
    hipLaunchKernelGGL(k_axpy_norm, dim3(grid), dim3(VEC_THREADS), 0, st, jobs_d, chunk_job_d, chunk_idx_d, n_chunks);
    return hipGetLastError();
}

// 16-byte loads need every vector (base + k ld) and y 16-byte aligned
static bool cgs_aligned(const double *basis, int64_t ld, const double *y) {
    return ((((uintptr_t)basis | (uintptr_t)y) & 15) == 0) && (ld & 1) == 0;
}

hipError_t launch_multidot(const double *basis, int64_t ld, int nvec, const double *y, int64_t n, double *partials,
                           int n_chunks, hipStream_t st, const double *gate) {
    const int grid = n_chunks < 1 ? 1 : (n_chunks < 65536 ? n_chunks : 65536);
    if (cgs_aligned(basis, ld, y))
        hipLaunchKernelGGL(k_multidot<true>, dim3(grid), dim3(CGS_THREADS), 0, st, basis, ld, nvec, y, n, partials,
                           n_chunks, gate);
    else
        hipLaunchKernelGGL(k_multidot<false>, dim3(grid), dim3(CGS_THREADS), 0, st, basis, ld, nvec, y, n, partials,
                           n_chunks, gate);
    return hipGetLastError();
}

hipError_t launch_multidot_reduce(const double *partials, int n_chunks, int nvec, const double *scale, double *coef,
                                  hipStream_t st, const double *gate) {
    hipLaunchKernelGGL(k_multidot_reduce, dim3(nvec), dim3(VEC_THREADS), 0, st, partials, n_chunks, scale, coef, gate);
    return hipGetLastError();
}

hipError_t launch_multiaxpy(const double *basis, int64_t ld, int nvec, const double *coef, const double *scale,
                            double *y, int64_t n, double *partials, int n_chunks, double sign, hipStream_t st,
                            const double *gate) {
    const int grid = n_chunks < 1 ? 1 : (n_chunks < 65536 ? n_chunks : 65536);
    if (cgs_aligned(basis, ld, y))
        hipLaunchKernelGGL(k_multiaxpy<true>, dim3(grid), dim3(CGS_THREADS), 0, st, basis, ld, nvec, coef, scale, y, n,
                           partials, n_chunks, sign, gate);
    else
        hipLaunchKernelGGL(k_multiaxpy<false>, dim3(grid), dim3(CGS_THREADS), 0, st, basis, ld, nvec, coef, scale, y,
                           n, partials, n_chunks, sign, gate);
    return hipGetLastError();
}

hipError_t launch_scale_copy(const double *x, double *y, int64_t n, double a, hipStream_t st) {
    int grid = (int)((n + 255) / 256);
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_scale_copy, dim3(grid), dim3(256), 0, st, x, y, n, a);
    return hipGetLastError();
}

hipError_t launch_fill_normal(double *y, int64_t n, uint64_t seed, hipStream_t st) {
    int grid = (int)((n + 255) / 256);
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_fill_normal, dim3(grid), dim3(256), 0, st, y, n, seed);
    return hipGetLastError();
}

}  // namespace ecut

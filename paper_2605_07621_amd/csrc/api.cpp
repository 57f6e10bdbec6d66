// C ABI of libecut: handle life cycle, device upload, H*psi, batched H*psi
// and the canonical <-> bipartite permutations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "ecut_internal.h"
#include "kernels.h"
#include "runtime.h"

static ecut_status check_dev(const ecut_sectors *s);   // handle on the current device

namespace ecut {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

ecut_status fail(ecut_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

ecut_status hip_fail(hipError_t e, const char *what) {
    return fail(ECUT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------- per-device resources
namespace {
struct DevRes {
    uint64_t *binom = nullptr;
    int n_cu = 0;
    size_t max_lds = 0;
    bool lds_set = false;
};
std::mutex g_dev_mu;
std::map<int, DevRes> g_dev;
}  // namespace

static std::atomic<size_t> g_last_max_lds{0};   // read by launches on any thread

ecut_status device_res(int *dev_out, const uint64_t **binom_out, int *n_cu_out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> g(g_dev_mu);
    DevRes &R = g_dev[dev];
    if (!R.binom) {
        std::vector<uint64_t> t(65 * 65);
        for (int n = 0; n <= 64; ++n)
            for (int k = 0; k <= 64; ++k) t[n * 65 + k] = binom(n, k);
        void *p = nullptr;
        e = hipMalloc(&p, t.size() * sizeof(uint64_t));
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(binomial table)");
        e = hipMemcpy(p, t.data(), t.size() * sizeof(uint64_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(binomial table)");
        R.binom = (uint64_t *)p;
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
        R.n_cu = prop.multiProcessorCount;
        R.max_lds = prop.sharedMemPerBlock;
        // Raising the dynamic-LDS cap is only a request: where the runtime
        // does not take the attribute, launches up to the device limit work
        // without it, so a refusal is cleared and ignored.
        e = set_hub_lds_limits((size_t)prop.sharedMemPerBlock > 65536 ? prop.sharedMemPerBlock : 65536);
        if (e != hipSuccess) (void)hipGetLastError();
        R.lds_set = e == hipSuccess;
    }
    if (dev_out) *dev_out = dev;
    if (binom_out) *binom_out = R.binom;
    if (n_cu_out) *n_cu_out = R.n_cu;
    g_last_max_lds = R.max_lds;
    return ECUT_OK;
}

// ---------------------------------------------------------------- upload
namespace {
struct Arena {
    size_t off = 0;
    struct Piece {
        size_t off;
        const void *src;
        size_t bytes;
    };
    std::vector<Piece> pieces;
    template <class T>
    size_t add(const std::vector<T> &v) {
        size_t o = off;
        size_t b = v.size() * sizeof(T);
        if (b) pieces.push_back({o, v.data(), b});
        off += (b + 255) & ~(size_t)255;
        if (b == 0) off += 256;   // keep a distinct, valid address
        return o;
    }
};
}  // namespace

// ---------------------------------------------------------------- table memory
// The sector tables of a handle come from the caller's allocator when one is
// set (ecut_set_allocator), else from hipMalloc.  Each allocation remembers
// the pair that made it, so it is released through that pair even after the
// caller installs another one.
namespace {
struct MetaAlloc {
    ecut_alloc_fn alloc = nullptr;
    ecut_free_fn free = nullptr;
    void *user = nullptr;
};
std::mutex g_alloc_mu;
MetaAlloc g_alloc;
std::map<void *, std::pair<MetaAlloc, size_t>> g_alloc_owner;   // live allocations of callers' allocators
}  // namespace

static ecut_status table_alloc(void **p, size_t bytes, int device) {
    MetaAlloc a;
    {
        std::lock_guard<std::mutex> g(g_alloc_mu);
        a = g_alloc;
    }
    if (!a.alloc) {
        const hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) return fail(ECUT_ENOMEM, std::string("hipMalloc(sector tables): ") + hipGetErrorString(e));
        return ECUT_OK;
    }
    void *m = a.alloc(bytes, device, a.user);
    if (!m) return fail(ECUT_ENOMEM, "the caller's allocator returned NULL for the sector tables");
    if ((uintptr_t)m & 255) {
        a.free(m, bytes, device, a.user);
        return fail(ECUT_EINVAL, "the caller's allocator returned memory that is not 256-byte aligned");
    }
    std::lock_guard<std::mutex> g(g_alloc_mu);
    g_alloc_owner[m] = {a, bytes};
    *p = m;
    return ECUT_OK;
}

static void table_free(void *p, int device) {
    MetaAlloc a;
    size_t bytes = 0;
    {
        std::lock_guard<std::mutex> g(g_alloc_mu);
        auto it = g_alloc_owner.find(p);
        if (it != g_alloc_owner.end()) {
            a = it->second.first;
            bytes = it->second.second;
            g_alloc_owner.erase(it);
        }
    }
    if (!a.free) {   // made by hipMalloc (the wait inside hipFree happens outside the lock)
        (void)hipFree(p);
        return;
    }
    // hipFree waits for the device; a caller's free may hand the memory out
    // again at once, so kernels still reading the tables must finish first
    (void)hipDeviceSynchronize();
    a.free(p, bytes, device, a.user);
}

void release_device(ecut_sectors *s) {
    if (s->dev_mem) {
        int cur = 0;
        hipGetDevice(&cur);
        if (s->device >= 0 && s->device != cur) (void)hipSetDevice(s->device);
        table_free(s->dev_mem, s->device >= 0 ? s->device : cur);
        if (s->device >= 0 && s->device != cur) (void)hipSetDevice(cur);
    }
    s->dev_mem = nullptr;
    s->on_device = false;
}

ecut_status upload(ecut_sectors *s) {
    int dev = 0;
    ecut_status st = device_res(&dev, nullptr, nullptr);
    if (st != ECUT_OK) return st;
    Arena A;
    const size_t o_blocks = A.add(s->blocks);
    const size_t o_lw = A.add(s->lwords), o_rw = A.add(s->rwords);
    const size_t o_hlp = A.add(s->hl_ptr), o_hlc = A.add(s->hl_col), o_hlv = A.add(s->hl_val);
    const size_t o_hrp = A.add(s->hr_ptr), o_hrc = A.add(s->hr_col), o_hrv = A.add(s->hr_val);
    const size_t o_dl = A.add(s->diag_l), o_dr = A.add(s->diag_r);
    const size_t o_xd = A.add(s->xdiag), o_xb = A.add(s->xbond), o_maps = A.add(s->maps), o_xdl = A.add(s->xdl);
    std::vector<ItemDev> row_items(std::max(s->items_cap, s->items.size()), ItemDev{0, 0, 0, 0, 0, 0});
    std::copy(s->items.begin(), s->items.end(), row_items.begin());   // capacity for any tile size
    const size_t o_items = A.add(row_items);
    size_t o_lc = 0, o_le = 0, o_lr = 0, o_hc = 0, o_he = 0, o_seg = 0, o_xbh = 0, o_cf = 0, o_u = 0, o_rw16 = 0,
           o_rw32 = 0, o_cor = 0, o_order = 0;
    if (s->hub_ok) {
        o_lc = A.add(s->hub_lo_cnt);
        o_le = A.add(s->hub_lo_ent);
        o_lr = A.add(s->hub_lo_rank);
        o_hc = A.add(s->hub_hi_cnt);
        o_he = A.add(s->hub_hi_ent);
        o_seg = A.add(s->hub_seg_off);
        o_xbh = A.add(s->hub_xb);
        o_cf = A.add(s->hub_coef);
        o_u = A.add(s->hub_u);
        o_rw16 = A.add(s->hub_rw16);
        o_rw32 = A.add(s->hub_rw32);
        o_cor = A.add(s->hub_col_of_rank);
        o_order = A.add(s->row_order);
    }
    size_t o_hcc = 0, o_hsc = 0, o_hhw = 0, o_hhc = 0, o_hhe = 0, o_hlw = 0, o_hlcn = 0, o_hle = 0, o_hit = 0;
    std::vector<HubItem> items_cap;   // must outlive the copies below
    if (s->hub_ok) {
        o_hcc = A.add(s->hc_cls);
        o_hsc = A.add(s->hc_segcol);
        o_hhw = A.add(s->hc_hiw);
        o_hhc = A.add(s->hc_hicnt);
        o_hhe = A.add(s->hc_hient);
        o_hlw = A.add(s->hc_low);
        o_hlcn = A.add(s->hc_locnt);
        o_hle = A.add(s->hc_loent);
        items_cap.assign(std::max(s->hub_items_cap, s->hub_items_ord.size()), HubItem{0, 0, 0, -1});
        std::copy(s->hub_items_ord.begin(), s->hub_items_ord.end(), items_cap.begin());
        o_hit = A.add(items_cap);
    }
    size_t o_srl = 0, o_srh = 0, o_sfm = 0, o_sfc = 0, o_hbm = 0, o_hbb = 0, o_hbc = 0;
    if (s->spin_ok || s->hubrow_ok || s->sp2_ok) {
        o_srl = A.add(s->spin_rank_lo);
        o_srh = A.add(s->spin_rank_hi);
    }
    if (s->hubrow_ok) {
        o_hbm = A.add(s->hrow_bmask);
        o_hbb = A.add(s->hrow_bbetw);
        o_hbc = A.add(s->hrow_bcoef);
    }
    size_t o_spr = 0, o_spb = 0, o_spp = 0, o_spc = 0, o_spv = 0, o_spt = 0, o_sptb = 0;
    if (s->spin_ok || s->sp2_ok) {
        o_sfm = A.add(s->spin_fmask);
        o_sfc = A.add(s->spin_fcoef);
        o_spr = A.add(s->sp_level_rows);
        o_spb = A.add(s->sp_lblocks);
        o_spp = A.add(s->sp_pptr);
        o_spc = A.add(s->sp_pcol);
        o_spv = A.add(s->sp_pval);
        o_spt = A.add(s->sp_tab);
        o_sptb = A.add(s->sp_tbase);
    }
    size_t o_3si = 0, o_3li = 0, o_3lo = 0, o_3hn = 0, o_3hc = 0;
    if (s->hub3_ok) {
        o_3si = A.add(s->h3_seginfo);
        o_3li = A.add(s->h3_loinfo);
        o_3lo = A.add(s->h3_looff);
        o_3hn = A.add(s->h3_hnb);
        o_3hc = A.add(s->h3_hcnt);
    }
    size_t o_5us = 0, o_5uh = 0, o_5ul = 0, o_5ux = 0, o_5it = 0;
    if (s->hubseg_ok) {
        o_5us = A.add(s->hs_useg);
        o_5uh = A.add(s->hs_uhnb);
        o_5ul = A.add(s->hs_ulo);
        o_5ux = A.add(s->hs_ucross);
        o_5it = A.add(s->hs_items);
    }
    size_t o_6k = 0, o_6v = 0, o_6r = 0, o_6p = 0, o_6c = 0, o_6w = 0;
    if (s->hub6_ok) {
        o_6k = A.add(s->h6_col);
        o_6v = A.add(s->h6_val);
        o_6r = A.add(s->level_rows);
        o_6p = A.add(s->h6_pptr);
        o_6c = A.add(s->h6_pcol);
        o_6w = A.add(s->h6_pval);
    }
    void *mem = nullptr;
    st = table_alloc(&mem, A.off, dev);
    if (st != ECUT_OK) return st;
    // one host image of the whole block, one copy (each copy of pageable
    // memory is a synchronous call with its own staging)
    std::vector<char> image(A.off, 0);
    for (auto &p : A.pieces) std::memcpy(image.data() + p.off, p.src, p.bytes);
    hipError_t e = hipMemcpy(mem, image.data(), A.off, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        table_free(mem, dev);
        return hip_fail(e, "hipMemcpy(sector tables)");
    }
    char *b = (char *)mem;
    ProblemDev &P = s->prob;
    P = ProblemDev{};
    P.kind = s->kind;
    P.n_blocks = (int32_t)s->blocks.size();
    P.n_xdiag = (int32_t)s->xdiag.size();
    P.n_xbond = (int32_t)s->xbond.size();
    P.blocks = (const BlockDev *)(b + o_blocks);
    P.lwords = (const uint32_t *)(b + o_lw);
    P.rwords = (const uint32_t *)(b + o_rw);
    P.hl_ptr = (const int32_t *)(b + o_hlp);
    P.hl_col = (const int32_t *)(b + o_hlc);
    P.hl_val = (const double *)(b + o_hlv);
    P.hr_ptr = (const int32_t *)(b + o_hrp);
    P.hr_col = (const int32_t *)(b + o_hrc);
    P.hr_val = (const double *)(b + o_hrv);
    P.diag_l = (const double *)(b + o_dl);
    P.diag_r = (const double *)(b + o_dr);
    P.xdiag = (const XDiagDev *)(b + o_xd);
    P.xdl = (const double *)(b + o_xdl);
    P.n_xr = (int32_t)s->xr_site.size();
    for (int g = 0; g < P.n_xr; ++g) P.xr_site[g] = s->xr_site[g];
    P.xr_lo = P.n_xr > 0 ? P.xr_site[0] : 0;
    P.xr_contig = 1;
    for (int g = 1; g < P.n_xr; ++g)
        if (P.xr_site[g] != P.xr_lo + g) P.xr_contig = 0;
    P.xbond = (const XBondDev *)(b + o_xb);
    P.maps = (const int32_t *)(b + o_maps);
    P.dim = s->dim;
    P.xscale = 1.0;
    if (s->spin_ok || s->sp2_ok) {
        P.spin_ok = (s->spin_ok && s->tune.variant == 0) ? 1 : 0;
        P.n_rflip = (int32_t)s->spin_fmask.size();
        P.max_d_r = s->max_d_r;
        P.rank_lo = (const int32_t *)(b + o_srl);
        P.rank_hi = (const int32_t *)(b + o_srh);
        P.rflip_mask = (const uint32_t *)(b + o_sfm);
        P.rflip_coef = (const double *)(b + o_sfc);
        s->dev_sp_rows = (int32_t *)(b + o_spr);
        s->dev_sp_lblocks = (SpinLBlock *)(b + o_spb);
        s->dev_sp_pptr = (const int32_t *)(b + o_spp);
        s->dev_sp_pcol = (const int32_t *)(b + o_spc);
        s->dev_sp_pval = (const double *)(b + o_spv);
        s->dev_sp_tab = (const uint16_t *)(b + o_spt);
        s->dev_sp_tbase = (const int64_t *)(b + o_sptb);
    }
    s->dev_items = (ItemDev *)(b + o_items);
    if (s->hub_ok) {
        HubDev &H = P.hub;
        H = s->hub;
        H.lo_cnt = (const int32_t *)(b + o_lc);
        H.lo_ent = (const int32_t *)(b + o_le);
        H.lo_rank = (const int32_t *)(b + o_lr);
        H.hi_cnt = (const int32_t *)(b + o_hc);
        H.hi_ent = (const int32_t *)(b + o_he);
        H.seg_off = (const int32_t *)(b + o_seg);
        H.xb = (const int32_t *)(b + o_xbh);
        H.coef = (const double *)(b + o_cf);
        H.u = (const double *)(b + o_u);
        H.rwords16 = s->hub_rw16.empty() ? nullptr : (const uint16_t *)(b + o_rw16);
        if (s->hubrow_ok) {
            H.n_dbond = (int32_t)s->hrow_bmask.size();
            H.dbond_mask = (const uint32_t *)(b + o_hbm);
            H.dbond_betw = (const uint32_t *)(b + o_hbb);
            H.dbond_coef = (const double *)(b + o_hbc);
            H.rank_lo = (const int32_t *)(b + o_srl);
            H.rank_hi = (const int32_t *)(b + o_srh);
        }
        H.rwords32 = (const uint32_t *)(b + o_rw32);
        H.col_of_rank = (const int32_t *)(b + o_cor);
        s->dev_row_order = (int32_t *)(b + o_order);
        H.cls = (const int32_t *)(b + o_hcc);
        H.cls_segcol = (const int32_t *)(b + o_hsc);
        H.cls_hiw = (const int32_t *)(b + o_hhw);
        H.cls_hicnt = (const int32_t *)(b + o_hhc);
        H.cls_hient = (const int32_t *)(b + o_hhe);
        H.cls_low = (const int32_t *)(b + o_hlw);
        H.cls_locnt = (const int32_t *)(b + o_hlcn);
        H.cls_loent = (const int32_t *)(b + o_hle);
        s->dev_hub_items = (HubItem *)(b + o_hit);
    }
    if (s->hub3_ok) {
        Hub3Args &A3 = s->h3;
        A3 = Hub3Args{};
        A3.hop = s->hub.hop0;
        A3.u0 = s->hub.u0;
        A3.hl_ptr = P.hl_ptr;
        A3.hl_col = P.hl_col;
        A3.hl_val = P.hl_val;
        A3.n_rows = s->blocks[0].d_l;
        A3.lwords = P.lwords;
        A3.cls = P.hub.cls;
        A3.seginfo = (const int4 *)(b + o_3si);
        A3.loinfo = (const int4 *)(b + o_3li);
        A3.looff = (const int32_t *)(b + o_3lo);
        A3.hnb = (const int32_t *)(b + o_3hn);
        A3.hcnt = (const int32_t *)(b + o_3hc);
        A3.items = s->dev_hub_items;
        A3.n_items = (int32_t)s->hub_items.size();
        A3.dR = s->blocks[0].d_r;
        A3.h = s->hub.h;
        A3.hs = s->h3_hs;
        A3.max_tile = s->h3_max_tile;
        A3.max_nseg = s->hub.max_nseg;
        A3.max_l = 0;
        for (size_t ci = 0; ci + 7 < s->hc_cls.size(); ci += 8) A3.max_l = std::max(A3.max_l, s->hc_cls[ci]);
    }
    if (s->hubseg_ok) {
        HubSegArgs &G = s->hseg;
        G = HubSegArgs{};
        G.hop = s->hub.hop0;
        G.u0 = s->hub.u0;
        G.lwords = P.lwords;
        G.cls = P.hub.cls;
        G.seginfo = (const int4 *)(b + o_3si);
        G.loinfo = (const int4 *)(b + o_3li);
        G.looff = (const int32_t *)(b + o_3lo);
        G.hnb = (const int32_t *)(b + o_3hn);
        G.hcnt = (const int32_t *)(b + o_3hc);
        G.useg = (const int4 *)(b + o_5us);
        G.uhnb = (const int32_t *)(b + o_5uh);
        G.ulo = (const int32_t *)(b + o_5ul);
        G.ucross = (const int32_t *)(b + o_5ux);
        G.items = (const HubSegItem *)(b + o_5it);
        G.n_items = (int32_t)s->hs_items.size();
        G.dR = s->blocks[0].d_r;
        G.h = s->hub.h;
        G.hs = s->h3_hs;
        G.uhs = s->hs_uhs;
    }
    if (s->hub6_ok) {
        const BlockDev &B0 = s->blocks[0];
        HubUArgs &U = s->h6u;
        U = HubUArgs{};
        // level order: a row's neighbours sit in the levels beside it; the
        // left operator's CSR in that order
        U.hl_ptr = (const int32_t *)(b + o_6p);
        U.hl_col = (const int32_t *)(b + o_6c);
        U.hl_val = (const double *)(b + o_6w);
        U.rows = (const int32_t *)(b + o_6r);
        U.uniform = 1;
        for (double v : s->hl_val) U.uniform = U.uniform && v == s->hl_val[0];
        U.hop = s->hl_val.empty() ? 0.0 : s->hl_val[0];
        U.n_rows = B0.d_l;
        U.dR = B0.d_r;
        HubDArgs &D = s->h6d;
        D = HubDArgs{};
        D.n_slots = s->h6_maxq;
        D.col = (const int32_t *)(b + o_6k);
        D.val = s->h6_uniform ? nullptr : (const double *)(b + o_6v);
        D.hop = s->h6_hop;
        D.lwords = P.lwords;
        D.rwords = P.hub.rwords32;
        D.u = P.hub.u;
        D.u0 = s->hub.u0;
        D.uniform_u = s->hub.uniform_u;
        D.n_rows = B0.d_l;
        D.dR = B0.d_r;
    }
    s->dev_mem = mem;
    s->dev_bytes = A.off;
    s->device = dev;
    s->on_device = true;
    return ECUT_OK;
}

int32_t max_tile_elems(const ecut_sectors *s) {
    int64_t m = 0;
    for (auto &it : s->items) m = std::max<int64_t>(m, (int64_t)(it.row1 - it.row0) * s->blocks[it.block].d_r);
    return (int32_t)m;
}

// Item counts of the two-pass kernels for the current tuning: the left pass
// takes `grid` rows of the level order (0 = HUBU_ROWS) per item over slabs of
// 64 lanes x 1 or 2 columns; the right pass `tile` rows (0 = HUBD_ROWS) x
// HUBD_THREADS columns per item.
static int32_t hub6_rows_d(const ecut_sectors *s) { return s->tune.tile > 0 ? s->tune.tile : HUBD_ROWS; }

void hub6_shape(const ecut_sectors *s, HubUArgs &U, HubDArgs &D) {
    const int32_t dR = s->blocks[0].d_r, nr = s->blocks[0].d_l;
    const int32_t cols = (dR % 2 == 0 ? 2 : 1) * 64;
    U.rows_per_item = s->tune.grid > 0 ? s->tune.grid : HUBU_ROWS;
    U.n_rgroups = (nr + U.rows_per_item - 1) / U.rows_per_item;
    U.slab_ways = (s->tune.variant == 7 && s->tune.tile > 0) ? s->tune.tile : 1;
    U.n_slabs = ((dR + cols - 1) / cols + U.slab_ways - 1) / U.slab_ways;
    U.n_items = U.n_slabs * U.n_rgroups;
    D.rows_per_item = hub6_rows_d(s);
    D.n_chunks = (dR + HUBD_THREADS - 1) / HUBD_THREADS;
    D.n_items = ((nr + D.rows_per_item - 1) / D.rows_per_item) * D.n_chunks;
}

// One application on a stream, with the Lanczos epilogue fields of `P`
// already filled in by the caller.
ecut_status launch_apply(const ecut_sectors *s, const ProblemDev &P, hipStream_t st) {
    int dev = 0, n_cu = 0;
    ecut_status rs = device_res(&dev, nullptr, &n_cu);
    if (rs != ECUT_OK) return rs;
    hipError_t e;
    if (s->kernel == 1) {
        const ApplyTuning &T = s->tune;
        const int n_xcd = T.n_xcd > 0 ? T.n_xcd : 8;
        if ((T.variant == 0 || T.variant == 3) && s->hub3_ok) {
            const size_t lds = hub3_lds_bytes(s);
            if (lds > g_last_max_lds) return fail(ECUT_EUNSUPPORTED, "class tiles exceed the device's LDS per work group");
            const int grid = T.grid > 0 ? T.grid : n_cu * hub_blocks_per_cu(3, lds);
            Hub3Args A3 = s->h3;
            A3.x = P.x;
            A3.y = P.y;
            A3.z = P.z;
            A3.partials = P.partials;
            A3.items = s->dev_hub_items;
            A3.n_items = (int32_t)s->hub_items_ord.size();
            A3.xscale = P.xscale;
            A3.zcoef = P.zcoef;
            A3.dscale = P.dscale;
            const int slab_grid = 8 * std::max(1, (n_cu / 8) * hub_blocks_per_cu(4, 0));
            e = launch_hub3(s, A3, grid, n_xcd, T.variant == 3, slab_grid, st);
        } else if ((T.variant == 6 && s->hub6_ok) || (T.variant == 7 && s->hub3_ok)) {
            // left operator on flat slab items of `grid` rows (0 = HUBU_ROWS)
            HubUArgs U = s->h6u;
            HubDArgs D = s->h6d;
            hub6_shape(s, U, D);
            U.x = D.x = P.x;
            U.y = D.y = P.y;
            e = launch_hub6_left(U, n_xcd, st);
            if (e == hipSuccess && T.variant == 6) {
                D.z = P.z;
                D.partials = P.partials;
                D.xscale = P.xscale;
                D.zcoef = P.zcoef;
                D.dscale = P.dscale;
                e = launch_hubD_only(D, n_xcd, st);
            } else if (e == hipSuccess) {
                // right operator, diagonal and epilogue on class tiles (the
                // left operator's sum is already in y)
                const size_t lds = hub3_lds_bytes(s);
                if (e == hipSuccess && lds > g_last_max_lds)
                    return fail(ECUT_EUNSUPPORTED, "class tiles exceed the device's LDS per work group");
                Hub3Args A3 = s->h3;
                A3.x = P.x;
                A3.y = P.y;
                A3.z = P.z;
                A3.partials = P.partials;
                A3.items = s->dev_hub_items;
                A3.n_items = (int32_t)s->hub_items_ord.size();
                A3.xscale = P.xscale;
                A3.zcoef = P.zcoef;
                A3.dscale = P.dscale;
                const int grid = n_cu * hub_blocks_per_cu(3, lds);
                if (e == hipSuccess) e = launch_hub3(s, A3, grid, n_xcd, true, 0, st);
            }
        } else if (T.variant == 5 && s->hubseg_ok) {
            const size_t lds = (size_t)s->hs_max_tile * 8;
            if (lds > g_last_max_lds) return fail(ECUT_EUNSUPPORTED, "segment tiles exceed the device's LDS per work group");
            const int grid = T.grid > 0 ? T.grid : n_cu * hub_blocks_per_cu(5, lds);
            HubSegArgs G = s->hseg;
            G.x = P.x;
            G.y = P.y;
            G.z = P.z;
            G.partials = P.partials;
            G.xscale = P.xscale;
            G.zcoef = P.zcoef;
            G.dscale = P.dscale;
            e = launch_hubseg(s, G, grid, n_xcd == 1 ? 1 : 8, st);
        } else if (T.variant == 4 && s->hubrow_ok) {
            if (((uintptr_t)P.x | (uintptr_t)P.y | (uintptr_t)P.z) & 15)
                return fail(ECUT_EINVAL, "the whole-row kernel needs 16-byte aligned vectors");
            e = launch_hubrow(s, P, s->dev_row_order, s->blocks[0].d_l, T.grid, n_xcd == 8 ? 8 : 1,
                              T.tile > 0 ? T.tile : 1024, n_cu, st);
        } else if ((T.variant == 0 || T.variant == 2) && s->hub2_ok) {
            const size_t lds = hub2_lds_bytes(s);
            if (lds > g_last_max_lds) return fail(ECUT_EUNSUPPORTED, "class tiles exceed the device's LDS per work group");
            const int grid = T.grid > 0 ? T.grid : n_cu * hub_blocks_per_cu(2, lds);
            e = launch_hub2(s, P, s->dev_hub_items, (int)s->hub_items_ord.size(), grid, n_xcd, st);
        } else {
            if (hub_lds_bytes(s) > g_last_max_lds)
                return fail(ECUT_EUNSUPPORTED, "Hubbard kernel tables exceed the device's LDS per work group");
            const int grid = T.grid > 0 ? T.grid : n_cu;
            e = launch_hub(s, P, s->dev_row_order, s->blocks[0].d_l, grid, n_xcd, st);
        }
    } else if (s->sp2_ok && s->tune.variant == 2) {
        SpinLArgs L{};
        L.x = P.x;
        L.y = P.y;
        L.hl_ptr = s->dev_sp_pptr;
        L.hl_col = s->dev_sp_pcol;
        L.hl_val = s->dev_sp_pval;
        L.rows = s->dev_sp_rows;
        L.blocks = s->dev_sp_lblocks;
        L.n_blocks = (int32_t)s->sp_lblocks.size();
        L.n_items = s->sp_lblocks.empty() ? 0
                                          : s->sp_lblocks.back().item0 +
                                                s->sp_lblocks.back().n_rgroups * s->sp_lblocks.back().n_slabs;
        L.rows_per_item = s->tune.grid > 0 ? s->tune.grid : HUBU_ROWS;
        e = launch_spin2(L, P, s->dev_sp_tab, s->dev_sp_tbase, s->dev_items, s->sp_n_one, (int)s->items.size(),
                         s->max_d_r, s->tune.n_xcd == 1 ? 1 : 8, s->hub_spatial, st);
    } else if (P.spin_ok) {
        int grid = s->tune.grid;
        if (s->tune.order == 1) grid = std::max(8, ((grid > 0 ? grid : 2048) / 8) * 8);   // keeps chunk c on XCD c
        e = launch_spin(nullptr, P, s->dev_items, (int)s->items.size(), max_tile_elems(s), s->max_d_r, grid, st);
    } else {
        e = launch_rows(nullptr, P, s->dev_items, (int)s->items.size(), max_tile_elems(s), st);
    }
    if (e != hipSuccess) return hip_fail(e, "kernel launch (apply_H)");
    return ECUT_OK;
}

bool own_launch(const ecut_sectors *s) { return s->kernel == 1 || (s->sp2_ok && s->tune.variant == 2); }

bool hub6_batchable(const ecut_sectors *s) {
    return s->kernel == 1 && s->hub6_ok && s->tune.variant == 6 && s->h6_maxq <= HUBD_BATCH_SLOTS;
}

void hub6_batch_add(HubBatch &b, const ecut_sectors *s, const ProblemDev &P) {
    HubUArgs U = s->h6u;
    HubDArgs D = s->h6d;
    hub6_shape(s, U, D);
    U.x = D.x = P.x;
    U.y = D.y = P.y;
    D.z = P.z;
    D.partials = P.partials;
    D.xscale = P.xscale;
    D.zcoef = P.zcoef;
    D.dscale = P.dscale;
    b.u.push_back(U);
    b.d.push_back(D);
    b.off_u.push_back(b.off_u.back() + U.n_items);
    b.off_d.push_back(b.off_d.back() + D.n_items);
}

HubBatchLayout hub6_batch_layout(const HubBatch &b, size_t base) {
    auto al = [](size_t o) { return (o + 255) & ~(size_t)255; };
    HubBatchLayout l;
    l.u = al(base);
    l.d = al(l.u + b.u.size() * sizeof(HubUArgs));
    l.off_u = al(l.d + b.d.size() * sizeof(HubDArgs));
    l.off_d = al(l.off_u + b.off_u.size() * sizeof(int32_t));
    l.bytes = l.off_d + b.off_d.size() * sizeof(int32_t);
    return l;
}

void hub6_batch_pack(const HubBatch &b, const HubBatchLayout &l, char *buf) {
    std::memcpy(buf + l.u, b.u.data(), b.u.size() * sizeof(HubUArgs));
    std::memcpy(buf + l.d, b.d.data(), b.d.size() * sizeof(HubDArgs));
    std::memcpy(buf + l.off_u, b.off_u.data(), b.off_u.size() * sizeof(int32_t));
    std::memcpy(buf + l.off_d, b.off_d.data(), b.off_d.size() * sizeof(int32_t));
}

hipError_t hub6_batch_launch(const HubBatch &b, const HubBatchLayout &l, const void *dev, hipStream_t st) {
    if (b.empty()) return hipSuccess;
    const char *d = (const char *)dev;
    return launch_hub6_batch((const HubUArgs *)(d + l.u), (const HubDArgs *)(d + l.d), (const int32_t *)(d + l.off_u),
                             (const int32_t *)(d + l.off_d), (int)b.u.size(), b.off_u.back(), b.off_d.back(), st);
}

// number of partial slots the apply kernel writes
int32_t apply_partial_slots(const ecut_sectors *s) {
    if (s->kernel != 1) return s->item_slots;
    if (s->tune.variant == 5 && s->hubseg_ok) return s->hs_n_slots;
    if (s->tune.variant == 7 && s->hub3_ok) return (int32_t)s->hub_items.size();
    if (s->tune.variant == 6 && s->hub6_ok) {
        HubUArgs U{};
        HubDArgs D{};
        hub6_shape(s, U, D);
        return D.n_items;
    }
    const bool tiles = ((s->tune.variant == 0 || s->tune.variant == 3) && (s->hub3_ok || s->hub2_ok)) ||
                       (s->tune.variant == 2 && s->hub2_ok);   // variants 1 and 4: one slot per row
    return tiles ? (int32_t)s->hub_items.size() : s->blocks[0].d_l;
}

// workspace size: either Hubbard variant may run on the same workspace
int32_t apply_partial_slots_max(const ecut_sectors *s) {
    // the two-pass kernels use the most slots with one row per right-pass item
    const int32_t h6 = s->hub6_ok ? s->blocks[0].d_l * ((s->blocks[0].d_r + HUBD_THREADS - 1) / HUBD_THREADS) : 0;
    return s->kernel == 1 ? std::max<int32_t>(std::max<int32_t>(std::max<int32_t>(s->blocks[0].d_l,
                                                                                    (int32_t)s->hub_items.size()),
                                                                  s->hubseg_ok ? s->hs_n_slots : 0),
                                              h6)
                          : std::max(s->item_slots_cap, s->item_slots);
}

// ---------------------------------------------------------------- staging buffers
ecut_status Staging::reserve(size_t bytes) {
    int cur = 0;
    hipGetDevice(&cur);
    if (device >= 0 && device != cur) release();
    if (bytes <= cap && dev) return ECUT_OK;
    ecut_status st = wait();
    if (st != ECUT_OK) return st;
    // kernels launched earlier may still read the old descriptors
    if (dev && hipDeviceSynchronize() != hipSuccess) return fail(ECUT_EDEVICE, "hipDeviceSynchronize(descriptor buffer)");
    if (dev) hipFree(dev);
    if (host) hipHostFree(host);
    dev = host = nullptr;
    cap = 0;
    size_t c = 4096;
    while (c < bytes) c *= 2;
    hipError_t e = hipMalloc(&dev, c);
    if (e != hipSuccess) return fail(ECUT_ENOMEM, "hipMalloc(descriptor buffer)");
    e = hipHostMalloc(&host, c, hipHostMallocDefault);
    if (e != hipSuccess) return fail(ECUT_ENOMEM, "hipHostMalloc(descriptor staging)");
    if (!ev) {
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    cap = c;
    device = cur;
    return ECUT_OK;
}

ecut_status Staging::wait() {
    if (pending && ev) {
        hipError_t e = hipEventSynchronize(ev);
        pending = false;
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(descriptor buffer)");
    }
    return ECUT_OK;
}

ecut_status Staging::upload(size_t bytes, hipStream_t st) {
    hipError_t e = hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(descriptors)");
    e = hipEventRecord(ev, st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    pending = true;
    return ECUT_OK;
}

void Staging::release() {
    if (pending && ev) hipEventSynchronize(ev);
    pending = false;
    if (dev) hipFree(dev);
    if (host) hipHostFree(host);
    if (ev) hipEventDestroy(ev);
    dev = host = nullptr;
    ev = nullptr;
    cap = 0;
    device = -1;
}

void make_rows_batch(const std::vector<ProblemDev> &probs, const std::vector<ItemDev> &items_in,
                     const std::vector<int32_t> &tiles, RowsBatch &b) {
    // the spin kernel takes the problems whose tuning selects it (as their
    // own ecut_apply_H does), the generic row kernel the others; the order
    // of the queue is kept within each group
    std::vector<ItemDev> items;
    items.reserve(items_in.size());
    b = RowsBatch{};
    for (const ItemDev &it : items_in)
        if (probs[it.prob].spin_ok) {
            items.push_back(it);
            b.spin_tile = std::max(b.spin_tile, tiles[it.prob]);
            b.spin_src = std::max(b.spin_src, probs[it.prob].max_d_r);
            if (b.first_spin < 0) b.first_spin = it.prob;
        }
    b.n_spin = (int)items.size();
    for (const ItemDev &it : items_in)
        if (!probs[it.prob].spin_ok) {
            items.push_back(it);
            b.rows_tile = std::max(b.rows_tile, tiles[it.prob]);
        }
    b.n_items = (int)items.size();
    b.pb = (probs.size() * sizeof(ProblemDev) + 255) & ~(size_t)255;
    b.buf.assign(b.pb + items.size() * sizeof(ItemDev), 0);
    std::memcpy(b.buf.data(), probs.data(), probs.size() * sizeof(ProblemDev));
    std::memcpy(b.buf.data() + b.pb, items.data(), items.size() * sizeof(ItemDev));
    if (b.first_spin >= 0) b.spin_single = probs[b.first_spin];
    if (!probs.empty()) b.rows_single = probs[0];
}

hipError_t launch_rows_batch(const RowsBatch &b, const void *dev, hipStream_t st) {
    const ProblemDev *probs_d = (const ProblemDev *)dev;
    const ItemDev *items_d = (const ItemDev *)((const char *)dev + b.pb);
    hipError_t e = hipSuccess;
    if (b.n_spin > 0) e = launch_spin(probs_d, b.spin_single, items_d, b.n_spin, b.spin_tile, b.spin_src, 0, st);
    if (e == hipSuccess && b.n_spin < b.n_items)
        e = launch_rows(probs_d, b.rows_single, items_d + b.n_spin, b.n_items - b.n_spin, b.rows_tile, st);
    return e;
}

ecut_status batch_launch_rows(const std::vector<ProblemDev> &probs, const std::vector<ItemDev> &items_in,
                              const std::vector<int32_t> &tiles, hipStream_t st) {
    static thread_local Staging S;
    RowsBatch b;
    make_rows_batch(probs, items_in, tiles, b);
    ecut_status rs = S.reserve(b.buf.size());
    if (rs != ECUT_OK) return rs;
    rs = S.wait();
    if (rs != ECUT_OK) return rs;
    std::memcpy(S.host, b.buf.data(), b.buf.size());
    hipError_t e = hipMemcpyAsync(S.dev, S.host, b.buf.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(batch descriptors)");
    e = launch_rows_batch(b, S.dev, st);
    if (e != hipSuccess) return hip_fail(e, "kernel launch (batched apply_H)");
    e = hipEventRecord(S.ev, st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    S.pending = true;
    return ECUT_OK;
}

ecut_status make_batch_plan(int32_t n, const ecut_sectors *const *s, const double *const *psi_d,
                            double *const *y_d, BatchPlan &pl) {
    if (n < 0 || (n > 0 && (!s || !psi_d || !y_d))) return fail(ECUT_EINVAL, "bad batch arguments");
    pl = BatchPlan{};
    if (n == 0) return ECUT_OK;
    std::vector<ProblemDev> probs(n);
    std::vector<ItemDev> items;
    std::vector<int32_t> tiles(n);
    for (int32_t k = 0; k < n; ++k) {
        ecut_status st = check_dev(s[k]);
        if (st != ECUT_OK) return st;
        if (!psi_d[k] || !y_d[k] || psi_d[k] == y_d[k]) return fail(ECUT_EINVAL, "bad vector in batch");
    }
    for (int32_t k = 0; k < n; ++k) {
        probs[k] = s[k]->prob;
        probs[k].x = psi_d[k];
        probs[k].y = y_d[k];
        probs[k].z = nullptr;
        probs[k].xscale = 1.0;
        probs[k].zcoef = 0.0;
        probs[k].partials = nullptr;
        tiles[k] = max_tile_elems(s[k]);
        if (hub6_batchable(s[k])) {
            hub6_batch_add(pl.hub, s[k], probs[k]);   // one merged launch per pass for all of them
        } else if (own_launch(s[k])) {
            pl.own.push_back(probs[k]);               // other Hubbard tunings and two-pass spin keep their own kernels
            pl.own_s.push_back(s[k]);
        } else {
            for (const ItemDev &it : s[k]->items) items.push_back(ItemDev{k, it.block, it.row0, it.row1, it.slot, 0});
        }
    }
    if (!items.empty()) {
        // one queue over all problems, largest tiles first (stable: problem order breaks ties)
        std::stable_sort(items.begin(), items.end(), [&](const ItemDev &a, const ItemDev &b) {
            const int64_t wa = (int64_t)(a.row1 - a.row0) * s[a.prob]->blocks[a.block].d_r;
            const int64_t wb = (int64_t)(b.row1 - b.row0) * s[b.prob]->blocks[b.block].d_r;
            return wa > wb;
        });
        make_rows_batch(probs, items, tiles, pl.rows);
        pl.has_rows = true;
        pl.buf = pl.rows.buf;
    }
    if (!pl.hub.empty()) {
        pl.hub_l = hub6_batch_layout(pl.hub, pl.buf.size());
        pl.buf.resize(pl.hub_l.bytes);
        hub6_batch_pack(pl.hub, pl.hub_l, pl.buf.data());
    }
    return ECUT_OK;
}

ecut_status launch_batch_plan(const BatchPlan &pl, const void *dev, hipStream_t st) {
    for (size_t k = 0; k < pl.own.size(); ++k) {
        ecut_status rs = launch_apply(pl.own_s[k], pl.own[k], st);
        if (rs != ECUT_OK) return rs;
    }
    hipError_t e = hipSuccess;
    if (pl.has_rows) e = launch_rows_batch(pl.rows, dev, st);
    if (e == hipSuccess) e = hub6_batch_launch(pl.hub, pl.hub_l, dev, st);
    if (e != hipSuccess) return hip_fail(e, "kernel launch (batched apply_H)");
    return ECUT_OK;
}

}  // namespace ecut

using namespace ecut;

// ---------------------------------------------------------------- ABI
extern "C" {

const char *ecut_last_error(void) { return g_err.c_str(); }

const char *ecut_version(void) { return "ecut 0.1 (gfx950)"; }

ecut_status ecut_set_allocator(ecut_alloc_fn alloc, ecut_free_fn free_fn, void *user) {
    if ((alloc == nullptr) != (free_fn == nullptr)) return fail(ECUT_EINVAL, "alloc and free must both be set or both be NULL");
    std::lock_guard<std::mutex> g(g_alloc_mu);
    g_alloc = MetaAlloc{alloc, free_fn, user};
    return ECUT_OK;
}

ecut_status ecut_build_sectors(const ecut_model_desc *model, const ecut_cut_desc *cut, ecut_qnum q, uint32_t flags,
                               ecut_sectors **out) {
    if (!out) return fail(ECUT_EINVAL, "out is NULL");
    *out = nullptr;
    if (flags & ~(uint32_t)ECUT_BUILD_HOST_ONLY) return fail(ECUT_EINVAL, "unknown flags");
    ecut_sectors *s = new (std::nothrow) ecut_sectors();
    if (!s) return fail(ECUT_ENOMEM, "host allocation");
    ecut_status st;
    try {
        st = build_host(model, cut, q, s);
    } catch (const std::bad_alloc &) {
        st = fail(ECUT_ENOMEM, "host allocation during sector build");
    }
    if (st == ECUT_OK && !(flags & ECUT_BUILD_HOST_ONLY)) st = upload(s);
    if (st != ECUT_OK) {
        delete s;
        return st;
    }
    *out = s;
    return ECUT_OK;
}

void ecut_sectors_free(ecut_sectors *s) {
    if (!s) return;
    release_device(s);
    delete s;
}

ecut_status ecut_sectors_get_info(const ecut_sectors *s, ecut_sectors_info *info) {
    if (!s || !info) return fail(ECUT_EINVAL, "null argument");
    ecut_sectors_info I{};
    I.dim = s->dim;
    I.n_blocks = (int32_t)s->blocks.size();
    I.n_left_sites = (int32_t)s->lsites.size();
    I.n_right_sites = (int32_t)s->rsites.size();
    I.max_d_r = s->max_d_r;
    I.n_cut_bonds = s->n_cut_bonds;
    I.n_cross_offdiag = 2 * (int32_t)s->xbond.size();
    I.n_cross_diag = (int32_t)s->xdiag.size();
    I.kernel = s->kernel;
    I.kernel_flags = (s->hub2_ok ? 1 : 0) | (s->hub3_ok ? 2 : 0) | (s->spin_ok ? 4 : 0) | (s->hubrow_ok ? 8 : 0) |
                     (s->hubseg_ok ? 16 : 0) | (s->hub6_ok ? 32 : 0) | (s->sp2_ok ? 64 : 0);
    I.device_bytes = (int64_t)s->dev_bytes;
    I.n_eff = s->n_eff;
    *info = I;
    return ECUT_OK;
}

ecut_status ecut_sectors_blocks(const ecut_sectors *s, int64_t *blocks) {
    if (!s || !blocks) return fail(ECUT_EINVAL, "null argument");
    for (size_t b = 0; b < s->blocks.size(); ++b) {
        const BlockDev &B = s->blocks[b];
        blocks[5 * b + 0] = B.q_l;
        blocks[5 * b + 1] = B.q_r;
        blocks[5 * b + 2] = B.d_l;
        blocks[5 * b + 3] = B.d_r;
        blocks[5 * b + 4] = B.offset;
    }
    return ECUT_OK;
}

ecut_status ecut_sectors_words(const ecut_sectors *s, int32_t block, uint32_t *l_words, uint32_t *r_words) {
    if (!s) return fail(ECUT_EINVAL, "null handle");
    if (block < 0 || block >= (int32_t)s->blocks.size()) return fail(ECUT_EINVAL, "block out of range");
    const BlockDev &B = s->blocks[block];
    if (l_words) std::memcpy(l_words, s->lwords.data() + B.lbase, sizeof(uint32_t) * (size_t)B.d_l);
    if (r_words) {
        if (s->hub_ok) std::memcpy(r_words, s->hub_rw32.data(), sizeof(uint32_t) * (size_t)B.d_r);   // column order
        else std::memcpy(r_words, s->rwords.data() + B.rbase, sizeof(uint32_t) * (size_t)B.d_r);
    }
    return ECUT_OK;
}

// Position and fermion sign of every canonical index of a spatial Hubbard
// cut, on the host's threads (the layout map of the device kernel).
static void hubsp_positions(const ecut_sectors *s, int64_t *pos, int8_t *sign) {
    const int nL = (int)s->lsites.size(), nR = (int)s->rsites.size();
    uint32_t lmask = 0, rmask = 0;
    for (int k : s->lsites) lmask |= 1u << k;
    for (int k : s->rsites) rmask |= 1u << k;
    const int64_t nd_words = (int64_t)binom(s->n_sites, s->n_dn);
    const int la0 = s->blocks.front().q_l, lb0 = s->blocks.front().q_l2;
    const int nb_b = s->blocks.back().q_l2 - lb0 + 1;
    auto compact = [](uint32_t w, uint32_t mask) {
        uint32_t out = 0;
        int k = 0;
        for (uint32_t m = mask; m; m &= m - 1u, ++k) out |= ((w >> __builtin_ctz(m)) & 1u) << k;
        return out;
    };
    auto work = [&](int64_t i0, int64_t i1) {
        for (int64_t i = i0; i < i1; ++i) {
            const uint32_t up = (uint32_t)colex_unrank(i / nd_words, s->n_up);
            const uint32_t dn = (uint32_t)colex_unrank(i % nd_words, s->n_dn);
            const uint32_t ul = compact(up, lmask), dl = compact(dn, lmask), ur = compact(up, rmask),
                           dr = compact(dn, rmask);
            const int a = __builtin_popcount(ul), b = __builtin_popcount(dl);
            const BlockDev &B = s->blocks[(size_t)((a - la0) * nb_b + (b - lb0))];
            const int64_t row = colex_rank(ul) * (int64_t)binom(nL, b) + colex_rank(dl);
            const int64_t col = colex_rank(ur) * (int64_t)binom(nR, s->n_dn - b) + colex_rank(dr);
            if (pos) pos[i] = B.offset + row * B.d_r + col;
            if (sign) {
                int par = __builtin_popcount(ur) * b;
                for (uint32_t m = lmask; m; m &= m - 1u) {
                    const uint32_t below = (m & (0u - m)) - 1u;
                    const int sb = __builtin_ctz(m);
                    if ((up >> sb) & 1u) par += __builtin_popcount(up & rmask & below);
                    if ((dn >> sb) & 1u) par += __builtin_popcount(dn & rmask & below);
                }
                sign[i] = (par & 1) ? -1 : 1;
            }
        }
    };
    const int64_t dim = s->dim;
    const unsigned hw = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
    const int64_t chunk = std::max<int64_t>(1 << 14, (dim + hw - 1) / hw);
    std::vector<std::thread> th;
    for (int64_t i0 = 0; i0 < dim; i0 += chunk) th.emplace_back(work, i0, std::min(dim, i0 + chunk));
    for (auto &t : th) t.join();
}

ecut_status ecut_canonical_signs(const ecut_sectors *s, int8_t *sign) {
    if (!s || !sign) return fail(ECUT_EINVAL, "null argument");
    if (s->hub_spatial) hubsp_positions(s, nullptr, sign);
    else std::fill(sign, sign + s->dim, (int8_t)1);
    return ECUT_OK;
}

ecut_status ecut_sectors_labels(const ecut_sectors *s, int32_t *labels) {
    if (!s || !labels) return fail(ECUT_EINVAL, "null argument");
    for (size_t b = 0; b < s->blocks.size(); ++b) {
        const BlockDev &B = s->blocks[b];
        labels[4 * b + 0] = B.q_l;
        labels[4 * b + 1] = B.q_l2;
        labels[4 * b + 2] = B.q_r;
        labels[4 * b + 3] = B.q_r2;
    }
    return ECUT_OK;
}

ecut_status ecut_canonical_positions(const ecut_sectors *s, int64_t *pos) {
    if (!s || !pos) return fail(ECUT_EINVAL, "null argument");
    if (s->hub_spatial) {
        hubsp_positions(s, pos, nullptr);
        return ECUT_OK;
    }
    if (s->kind == ECUT_HUBBARD) {
        // canonical index = up rank * d_R + down rank (up-major integer order)
        const int64_t dR = s->blocks[0].d_r;
        for (int64_t i = 0; i < s->dim; ++i) pos[i] = (i / dR) * dR + hub_column(s, i % dR);
        return ECUT_OK;
    }
    // Chunks of the canonical order on the host's threads: each chunk unranks
    // its first word and steps to the next word of the same popcount (the
    // smallest larger one: move the lowest movable set bit up by one and put
    // the set bits below it back at the bottom).
    const int qmin = s->blocks[0].q_l;
    const int64_t dim = s->dim;
    const unsigned hw = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
    const int64_t chunk = std::max<int64_t>(1 << 16, (dim + hw - 1) / hw);
    auto work = [&](int64_t i0, int64_t i1) {
        uint64_t w = colex_unrank(i0, s->n_up);
        for (int64_t i = i0; i < i1; ++i) {
            uint64_t l = 0, r = 0;
            for (size_t k = 0; k < s->lsites.size(); ++k) l |= ((w >> s->lsites[k]) & 1ull) << k;
            for (size_t k = 0; k < s->rsites.size(); ++k) r |= ((w >> s->rsites[k]) & 1ull) << k;
            const BlockDev &B = s->blocks[__builtin_popcountll(l) - qmin];
            pos[i] = B.offset + colex_rank(l) * B.d_r + colex_rank(r);
            if (w != 0 && i + 1 < i1) {
                const int t = __builtin_ctzll(w);                  // lowest set bit
                const int run = __builtin_ctzll(~(w >> t));        // set bits from there up
                w = (w & ~(((1ull << run) - 1) << t)) | (1ull << (t + run)) | ((1ull << (run - 1)) - 1);
            }
        }
    };
    std::vector<std::thread> th;
    for (int64_t i0 = 0; i0 < dim; i0 += chunk) th.emplace_back(work, i0, std::min(dim, i0 + chunk));
    for (auto &t : th) t.join();
    return ECUT_OK;
}

static ecut_status check_dev(const ecut_sectors *s) {
    if (!s) return fail(ECUT_EINVAL, "null handle");
    if (!s->on_device) return fail(ECUT_EINVAL, "handle was built with ECUT_BUILD_HOST_ONLY");
    int cur = -1;
    hipGetDevice(&cur);
    if (cur != s->device) return fail(ECUT_EINVAL, "handle lives on another device");
    return ECUT_OK;
}

static HubSpPerm hubsp_perm(const ecut_sectors *s, const uint64_t *binom_d) {
    HubSpPerm A{};
    A.blocks = s->prob.blocks;
    A.binom = binom_d;
    A.dim = s->dim;
    A.n_dn_words = (int64_t)binom(s->n_sites, s->n_dn);
    for (int k : s->lsites) A.lmask |= 1u << k;
    for (int k : s->rsites) A.rmask |= 1u << k;
    A.n_up = s->n_up;
    A.n_dn = s->n_dn;
    A.nL = (int32_t)s->lsites.size();
    A.nR = (int32_t)s->rsites.size();
    A.la0 = s->blocks.front().q_l;
    A.lb0 = s->blocks.front().q_l2;
    A.nb_b = s->blocks.back().q_l2 - A.lb0 + 1;
    return A;
}

static ecut_status permute(const ecut_sectors *s, const double *in, double *out, bool to_bip, void *stream) {
    ecut_status st = check_dev(s);
    if (st != ECUT_OK) return st;
    if (!in || !out) return fail(ECUT_EINVAL, "null vector");
    if (in == out) return fail(ECUT_EINVAL, "in and out must differ");
    hipStream_t hs = (hipStream_t)stream;
    hipError_t e;
    if (s->hub_spatial) {
        const uint64_t *bt = nullptr;
        st = device_res(nullptr, &bt, nullptr);
        if (st != ECUT_OK) return st;
        e = launch_perm_hubsp(hubsp_perm(s, bt), in, out, to_bip, hs);
    } else if (s->kind == ECUT_HUBBARD && s->hub_ok) {
        e = launch_perm_cols(s->prob.hub.col_of_rank, s->blocks[0].d_l, s->blocks[0].d_r, in, out, to_bip, hs);
    } else if (s->kind == ECUT_HUBBARD) {
        e = hipMemcpyAsync(out, in, sizeof(double) * (size_t)s->dim, hipMemcpyDeviceToDevice, hs);
    } else {
        const uint64_t *bt = nullptr;
        st = device_res(nullptr, &bt, nullptr);
        if (st != ECUT_OK) return st;
        e = launch_perm(s, bt, s->prob.blocks, in, out, to_bip, hs);
    }
    if (e != hipSuccess) return hip_fail(e, to_bip ? "ecut_import" : "ecut_export");
    return ECUT_OK;
}

ecut_status ecut_apply_cdag(const ecut_sectors *src, const ecut_sectors *dst, int32_t site, int32_t spin,
                            int32_t dagger, const double *x_d, double *y_d, void *stream) {
    ecut_status st = check_dev(src);
    if (st == ECUT_OK) st = check_dev(dst);
    if (st != ECUT_OK) return st;
    if (!x_d || !y_d || (const double *)y_d == x_d) return fail(ECUT_EINVAL, "null or overlapping vectors");
    if (src->kind != ECUT_HUBBARD || dst->kind != ECUT_HUBBARD || src->cut_kind != ECUT_CUT_UPDN ||
        dst->cut_kind != ECUT_CUT_UPDN)
        return fail(ECUT_EUNSUPPORTED, "c+ / c is built for Hubbard sectors with the up/down cut");
    if (src->n_sites != dst->n_sites) return fail(ECUT_EINVAL, "the two sectors belong to lattices of different size");
    if (site < 0 || site >= src->n_sites || spin < 0 || spin > 1) return fail(ECUT_EINVAL, "site or spin out of range");
    const int d = dagger ? 1 : -1;
    const int want_up = src->n_up + (spin == 0 ? d : 0), want_dn = src->n_dn + (spin == 1 ? d : 0);
    if (dst->n_up != want_up || dst->n_dn != want_dn)
        return fail(ECUT_EINVAL, "the destination sector must hold the source's particles with one more (c+) or one "
                                 "fewer (c) of the given spin");
    const uint64_t *bt = nullptr;
    st = device_res(nullptr, &bt, nullptr);
    if (st != ECUT_OK) return st;
    CdagArgs A{};
    A.x = x_d;
    A.y = y_d;
    A.dim = dst->dim;
    A.dR_dst = dst->blocks[0].d_r;
    A.dR_src = src->blocks[0].d_r;
    A.dst_lwords = dst->prob.lwords;
    A.dst_rwords = dst->hub_ok ? dst->prob.hub.rwords32 : dst->prob.rwords;
    A.src_col_of_rank = src->hub_ok ? src->prob.hub.col_of_rank : nullptr;
    A.binom = bt;
    A.site = site;
    A.spin = spin;
    A.dagger = dagger ? 1 : 0;
    if (A.dim == 0) return ECUT_OK;
    const hipError_t e = launch_cdag(A, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch (apply_cdag)");
    return ECUT_OK;
}

ecut_status ecut_import(const ecut_sectors *s, const double *canon_d, double *bip_d, void *stream) {
    return permute(s, canon_d, bip_d, true, stream);
}

ecut_status ecut_export(const ecut_sectors *s, const double *bip_d, double *canon_d, void *stream) {
    return permute(s, bip_d, canon_d, false, stream);
}

ecut_status ecut_apply_H(const ecut_sectors *s, const double *psi_d, double *y_d, void *stream) {
    ecut_status st = check_dev(s);
    if (st != ECUT_OK) return st;
    if (!psi_d || !y_d) return fail(ECUT_EINVAL, "null vector");
    if (psi_d == y_d) return fail(ECUT_EINVAL, "psi and y must not overlap");
    ProblemDev P = s->prob;
    P.x = psi_d;
    P.y = y_d;
    P.z = nullptr;
    P.xscale = 1.0;
    P.zcoef = 0.0;
    P.partials = nullptr;
    return launch_apply(s, P, (hipStream_t)stream);
}

ecut_status ecut_apply_H_batch(int32_t n, const ecut_sectors *const *s, const double *const *psi_d,
                               double *const *y_d, void *stream) {
    BatchPlan pl;
    ecut_status st = make_batch_plan(n, s, psi_d, y_d, pl);
    if (st != ECUT_OK || n == 0) return st;
    // a descriptor buffer whose previous batch has been copied (a ring of a
    // few per thread, so the call waits only when all of them are in flight)
    static thread_local Staging ring[4];
    static thread_local int next = 0;
    Staging *S = nullptr;
    for (int k = 0; k < 4 && !S; ++k) {
        Staging &c = ring[(next + k) % 4];
        if (!c.pending || hipEventQuery(c.ev) == hipSuccess) S = &c;
    }
    if (!S) S = &ring[next % 4];   // every buffer busy: the oldest use is waited for
    next = (int)(S - ring + 1) % 4;
    if (!pl.buf.empty()) {
        st = S->reserve(pl.buf.size());
        if (st == ECUT_OK) st = S->wait();
        if (st != ECUT_OK) return st;
        std::memcpy(S->host, pl.buf.data(), pl.buf.size());
        hipError_t e = hipMemcpyAsync(S->dev, S->host, pl.buf.size(), hipMemcpyHostToDevice, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(batch descriptors)");
    }
    st = launch_batch_plan(pl, S->dev, (hipStream_t)stream);
    if (st != ECUT_OK) return st;
    if (!pl.buf.empty()) {
        hipError_t e = hipEventRecord(S->ev, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        S->pending = true;
    }
    return ECUT_OK;
}

}  // extern "C"

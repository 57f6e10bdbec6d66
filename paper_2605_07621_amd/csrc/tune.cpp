// Launch tuning of ecut_apply_H and the autotuner.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "ecut_internal.h"
#include "runtime.h"

namespace ecut {
namespace {

std::mutex g_cache_mu;

}  // namespace

std::string tune_shape_key(const ecut_sectors *s) {
    hipDeviceProp_t prop;
    int dev = 0;
    hipGetDevice(&dev);
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    std::ostringstream k;
    k << arch << "/k" << s->kernel << "/s" << s->n_sites << "/u" << s->n_up << "/d" << s->n_dn << "/b"
      << s->blocks.size() << "/dim" << s->dim;
    return k.str();
}

namespace {

// The cache file is a flat JSON object {"key": [grid, n_xcd, row_order, variant, tile], ...};
// entries without the tile take the default tile.
std::map<std::string, ApplyTuning> read_cache(const char *path) {
    std::map<std::string, ApplyTuning> out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    size_t p = 0;
    while ((p = t.find('"', p)) != std::string::npos) {
        const size_t q = t.find('"', p + 1);
        if (q == std::string::npos) break;
        const std::string key = t.substr(p + 1, q - p - 1);
        const size_t a = t.find('[', q), b = t.find(']', q);
        if (a == std::string::npos || b == std::string::npos) break;
        ApplyTuning T{};
        const int got = std::sscanf(t.substr(a + 1, b - a - 1).c_str(), "%d , %d , %d , %d , %d", &T.grid, &T.n_xcd,
                                    &T.order, &T.variant, &T.tile);
        if (got == 4 || got == 5) out[key] = T;
        p = b;
    }
    return out;
}

void write_cache(const char *path, const std::map<std::string, ApplyTuning> &m) {
    std::ofstream f(path);
    f << "{\n";
    size_t k = 0;
    for (auto &kv : m) {
        f << "  \"" << kv.first << "\": [" << kv.second.grid << ", " << kv.second.n_xcd << ", " << kv.second.order
          << ", " << kv.second.variant << ", " << kv.second.tile << "]" << (++k < m.size() ? "," : "") << "\n";
    }
    f << "}\n";
}

ecut_status apply_tuning(ecut_sectors *s, const ApplyTuning &T) {
    if (T.order < 0 || T.order > 10 || T.grid < 0 || T.n_xcd < 0 || T.variant < 0 || T.variant > 7)
        return fail(ECUT_EINVAL, "bad tuning");
    if (s->kernel != 1 && T.variant > (s->spin_ok || s->sp2_ok ? 2 : 1))
        return fail(ECUT_EINVAL, "spin problems take variant 0, 1 or 2, generic problems 0 or 1 (2 with two-pass tables)");
    if (s->kernel != 1 && T.variant == 2) {
        if (!s->sp2_ok)
            return fail(ECUT_EUNSUPPORTED, "two-pass row kernels need at most 64 left-operator terms per row");
        if (T.grid > HUBU_RMAX * (HUBU_THREADS / 64))
            return fail(ECUT_EINVAL, "left-pass items of the two-pass row kernels take at most 32 rows");
    }
    if (T.tile < 0) return fail(ECUT_EINVAL, "tile must not be negative");
    if (s->spin_ok) {
        if (T.tile > SPIN_MANY_TILE) return fail(ECUT_EINVAL, "tile must lie in 0..512");
    } else if (s->kernel == 1 && T.variant == 4) {
        // the whole-row Hubbard kernel: tile = threads per work group
        if (T.tile != 0 && T.tile != 256 && T.tile != 512 && T.tile != 1024)
            return fail(ECUT_EINVAL, "whole-row work groups take 256, 512 or 1024 threads");
        if (T.tile != 0 && !s->blocks.empty() && s->blocks[0].d_r > 2 * HUBROW_P * T.tile)
            return fail(ECUT_EUNSUPPORTED, "rows longer than 14 columns per thread of the work group");
    } else if (s->kernel == 1 && (T.variant == 6 || T.variant == 7)) {
        // the two-pass kernels: tile = rows per item of the right-operator pass
        if (T.tile != 0 && T.tile != 1 && T.tile != 2 && T.tile != 4 && T.tile != 8 && T.tile != 16)
            return fail(ECUT_EINVAL, "two-pass items take 1, 2, 4, 8 or 16 rows");
        const int ways = (T.variant == 7 && T.tile > 0) ? T.tile : 1;
        if (T.grid > HUBU_RMAX * (HUBU_THREADS / 64) / ways)
            return fail(ECUT_EINVAL, "left-operator items take at most 32 rows (8 with 4 slabs side by side)");
    } else if (T.tile != 0) {
        return fail(ECUT_EUNSUPPORTED,
                    "the tile applies to the spin kernel, the whole-row and the two-pass Hubbard kernels only");
    }
    if (s->spin_ok && T.order > 1) return fail(ECUT_EINVAL, "spin problems take row order 0 or 1");
    if ((T.variant == 0 || T.variant == 2) && s->kernel == 1 && !s->hub2_ok)
        return fail(ECUT_EUNSUPPORTED, "class tiles not available");
    if (T.variant == 3 && s->kernel == 1 && !s->hub3_ok) return fail(ECUT_EUNSUPPORTED, "split passes not available");
    if (T.variant == 5 && s->kernel == 1 && !s->hubseg_ok)
        return fail(ECUT_EUNSUPPORTED, "segment tiles not available (needs uniform, sign-free hopping, <= 16 sites)");
    if (T.variant == 6 && s->kernel == 1 && !s->hub6_ok) return fail(ECUT_EUNSUPPORTED, "two-pass kernels not available");
    if (T.variant == 7 && s->kernel == 1 && !s->hub3_ok)
        return fail(ECUT_EUNSUPPORTED, "two passes with class tiles need the uniform-chain tables");
    if (T.variant == 7 && T.tile != 0 && T.tile != 1 && T.tile != 2 && T.tile != 4)
        return fail(ECUT_EINVAL, "variant 7 takes tile 0, 1, 2 or 4 (slabs side by side in a left-pass item)");
    if (T.variant == 4 && s->kernel == 1 && !s->hubrow_ok)
        return fail(ECUT_EUNSUPPORTED, "whole-row kernel not available (more than 16 sites, odd or too long rows)");
    if (s->kernel == 1 && (T.order != s->tune.order || T.variant != s->tune.variant)) {
        make_row_order(s, row_order_kind(T.order), s->row_order);
        make_hub_item_order(s, T.order, s->hub_items_ord);
        if (s->on_device && s->dev_row_order) {
            hipError_t e = hipMemcpy(s->dev_row_order, s->row_order.data(), s->row_order.size() * sizeof(int32_t),
                                     hipMemcpyHostToDevice);
            if (s->hub_items_ord.size() > s->hub_items_cap) return fail(ECUT_EINVAL, "work list exceeds its buffer");
            if (e == hipSuccess && s->dev_hub_items)
                e = hipMemcpy(s->dev_hub_items, s->hub_items_ord.data(), s->hub_items_ord.size() * sizeof(HubItem),
                              hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy(work order)");
        }
    }
    const int32_t tile = T.tile > 0 ? T.tile : SPIN_MANY_TILE, cur = s->tune.tile > 0 ? s->tune.tile : SPIN_MANY_TILE;
    const int32_t spin_order = T.variant == 2 ? 2 : T.order, cur_order = s->tune.variant == 2 ? 2 : s->tune.order;
    if (s->spin_ok && (tile != cur || spin_order != cur_order)) {
        std::vector<ItemDev> items;
        const int32_t slots = make_spin_items(s, tile, spin_order, items);
        if (items.size() > s->items_cap || slots > s->item_slots_cap)
            return fail(ECUT_EINVAL, "work list exceeds its buffer");
        if (s->on_device && s->dev_items) {
            hipError_t e =
                hipMemcpy(s->dev_items, items.data(), items.size() * sizeof(ItemDev), hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy(work items)");
        }
        s->items.swap(items);
        s->item_slots = slots;
    }
    if (s->hub_spatial && s->sp2_ok && (T.variant == 2) != (s->tune.variant == 2)) {
        // every row its own item for the two-pass kernels, else the row kernel's tiles
        std::vector<ItemDev> items;
        const int32_t slots = T.variant == 2 ? make_spin_items(s, 1, 2, items)
                                             : (items = s->generic_items, (int32_t)items.size());
        if (items.size() > s->items_cap || slots > s->item_slots_cap)
            return fail(ECUT_EINVAL, "work list exceeds its buffer");
        if (s->on_device && s->dev_items) {
            hipError_t e =
                hipMemcpy(s->dev_items, items.data(), items.size() * sizeof(ItemDev), hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy(work items)");
        }
        s->items.swap(items);
        s->item_slots = slots;
    }
    if (s->spin_ok || s->sp2_ok) {
        s->sp_n_one = 0;
        if (spin_order == 2)
            for (const ItemDev &it : s->items) s->sp_n_one += (it.row1 - it.row0 == 1) ? 1 : 0;
        const int32_t rpi = T.grid > 0 ? T.grid : HUBU_ROWS, cur_rpi = s->tune.grid > 0 ? s->tune.grid : HUBU_ROWS;
        if (T.variant == 2 && (rpi != cur_rpi || s->tune.variant != 2)) {
            std::vector<SpinLBlock> lb;
            spin_left_blocks(s, rpi, lb);
            if (lb.size() != s->sp_lblocks.size()) return fail(ECUT_EINVAL, "left-pass block table changed size");
            if (s->on_device && s->dev_sp_lblocks) {
                hipError_t e =
                    hipMemcpy(s->dev_sp_lblocks, lb.data(), lb.size() * sizeof(SpinLBlock), hipMemcpyHostToDevice);
                if (e != hipSuccess) return hip_fail(e, "hipMemcpy(left-pass blocks)");
            }
            s->sp_lblocks.swap(lb);
        }
    }
    s->tune = T;
    if (s->kernel != 1) s->prob.spin_ok = (s->spin_ok && s->on_device && T.variant == 0) ? 1 : 0;
    return ECUT_OK;
}

}  // namespace
}  // namespace ecut

using namespace ecut;

extern "C" {

ecut_status ecut_get_tuning(const ecut_sectors *s, ecut_tuning *t) {
    if (!s || !t) return fail(ECUT_EINVAL, "null argument");
    t->grid = s->tune.grid;
    t->n_xcd = s->tune.n_xcd;
    t->row_order = s->tune.order;
    t->variant = s->tune.variant;
    t->tile = s->tune.tile;
    return ECUT_OK;
}

ecut_status ecut_set_tuning(ecut_sectors *s, const ecut_tuning *t) {
    if (!s || !t) return fail(ECUT_EINVAL, "bad argument");
    ApplyTuning T{t->grid, t->n_xcd, t->row_order, t->variant, t->tile};
    return apply_tuning(s, T);
}

ecut_status ecut_autotune(ecut_sectors *s, const double *x_d, double *y_d, void *stream, ecut_tuning *best) {
    if (!s || !x_d || !y_d || x_d == y_d) return fail(ECUT_EINVAL, "bad argument");
    if (!s->on_device) return fail(ECUT_EINVAL, "handle was built with ECUT_BUILD_HOST_ONLY");
    hipStream_t st = (hipStream_t)stream;
    const char *cache_path = std::getenv("ECUT_TUNE_CACHE");
    const std::string key = tune_shape_key(s);
    if (cache_path) {
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto m = read_cache(cache_path);
        auto it = m.find(key);
        // an entry this problem cannot take (another model of the same
        // shape) is timed afresh
        if (it != m.end() && apply_tuning(s, it->second) == ECUT_OK) {
            if (best) ecut_get_tuning(s, best);
            return ECUT_OK;
        }
    }
    std::vector<ApplyTuning> cands;
    if (s->kernel == 1) {
        if (s->hub2_ok)
            for (int order = 0; order < 6; ++order)
                for (int xcd : {1, 8}) cands.push_back(ApplyTuning{0, xcd, order, 0});
        if (s->hub3_ok)
            for (int order : {6, 7, 8, 9, 10}) cands.push_back(ApplyTuning{0, 8, order, 0});
        if (s->hub3_ok)
            for (int order : {0, 1}) cands.push_back(ApplyTuning{0, 1, order, 3});
        for (int order : {0, 2})
            for (int xcd : {1, 8}) cands.push_back(ApplyTuning{0, xcd, order, 1});
        if (s->hubrow_ok)
            for (int threads : {1024, 512, 256})
                if (threads == 1024 || s->blocks[0].d_r <= 2 * HUBROW_P * threads)
                    for (int order : {0, 1, 2, 9})
                        for (int xcd : {1, 8}) cands.push_back(ApplyTuning{0, xcd, order, 4, threads == 1024 ? 0 : threads});
        if (s->hubseg_ok)
            for (int xcd : {1, 8}) cands.push_back(ApplyTuning{0, xcd, 0, 5});
        if (s->hub6_ok)
            for (int order : {0, 1, 2})
                for (int xcd : {1, 8})
                    for (int urows : {4, 8})
                        for (int rows : {2, 8}) cands.push_back(ApplyTuning{urows, xcd, order, 6, rows});
        if (s->hub3_ok)
            for (int urows : {4, 8})
                for (int order : {7, 8}) cands.push_back(ApplyTuning{urows, 8, order, 7, 0});
    } else if (s->spin_ok) {
        // spin kernel: short-row tile and grid; then the generic row kernel
        for (int order : {0, 1})
            for (int tile : {128, 256, 512})
                for (int grid : {0, 512, 1024}) cands.push_back(ApplyTuning{grid, 0, order, 0, tile});
        cands.push_back(ApplyTuning{0, 0, 0, 1, 0});
        // two-pass kernels: left-pass rows per item, XCD dealing
        if (s->sp2_ok)
            for (int rows : {4, 8, 16})
                for (int xcd : {1, 8}) cands.push_back(ApplyTuning{rows, xcd, 0, 2, 0});
    } else {
        cands.push_back(ApplyTuning{0, 0, 0, 0, 0});
        if (s->sp2_ok)   // the spatial Hubbard cut: the two-pass row kernels
            for (int rows : {4, 8, 16})
                for (int xcd : {1, 8}) cands.push_back(ApplyTuning{rows, xcd, 0, 2, 0});
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(ECUT_EDEVICE, "hipEventCreate");
    ProblemDev P = s->prob;
    P.x = x_d;
    P.y = y_d;
    P.z = nullptr;
    P.xscale = 1.0;
    P.zcoef = 0.0;
    P.partials = nullptr;
    float best_ms = 1e30f;
    ApplyTuning best_t = s->tune;
    ecut_status rs = ECUT_OK;
    for (const ApplyTuning &T : cands) {
        rs = apply_tuning(s, T);
        if (rs != ECUT_OK) break;
        P.spin_ok = s->prob.spin_ok;   // the kernel choice of this candidate
        rs = launch_apply(s, P, st);   // warm-up
        if (rs != ECUT_OK) break;
        hipEventRecord(e0, st);
        const int reps = 3;
        for (int r = 0; r < reps && rs == ECUT_OK; ++r) rs = launch_apply(s, P, st);
        hipEventRecord(e1, st);
        if (rs != ECUT_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess) { rs = fail(ECUT_EDEVICE, "autotune timing"); break; }
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
        if (ms < best_ms) { best_ms = ms; best_t = T; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rs != ECUT_OK) return rs;
    rs = apply_tuning(s, best_t);
    if (rs != ECUT_OK) return rs;
    if (cache_path) {
        std::lock_guard<std::mutex> g(g_cache_mu);
        auto m = read_cache(cache_path);
        m[key] = best_t;
        write_cache(cache_path, m);
    }
    if (best) ecut_get_tuning(s, best);
    return ECUT_OK;
}

}  // extern "C"

// Lanczos ground-state solver on the device (Paige's ordering):
//   u = H v_j - beta_{j-1} v_{j-1}, alpha_j = <v_j, u>   (fused into H*psi)
//   w = u - alpha_j v_j, beta_j = |w|                    (one fused pass)
//   optional classical Gram-Schmidt against all stored vectors, with a
//   second pass when the first loses more than half the squared norm
// Vectors are kept unnormalised (v_j = s_j w_j) so no scaling pass is needed;
// the scales enter the next H*psi and the updates as factors, which a small
// kernel derives from beta_j on the device, so the host need not answer
// before the next step is launched: three-term solves keep two steps in
// flight and the host processes step j while step j + 1 runs.  On the host,
// every step takes the lowest Ritz value of the tridiagonal matrix by Sturm
// bisection from the previous one (O(m)) and its eigenvector by inverse
// iteration for the residual beta_j |u_j|; implicit QL on the final matrix
// cross-checks the energy.
#include "lanczos.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>

#include "kernels.h"
#include "tridiag.h"

namespace ecut {

// Elements per norm partial: VEC_CHUNK with reorthogonalisation (its kernels
// share that layout); for three-term solves smaller, down to 1024, so a
// short vector's update pass still spreads over many work groups.
static int64_t chunk_of(int64_t n, bool reorth) {
    if (reorth) return VEC_CHUNK;
    int64_t c = 1024;
    while (c < VEC_CHUNK && c * 2048 < n) c *= 2;
    return c;
}
static int64_t n_chunks_of(int64_t n, bool reorth) {
    const int64_t c = chunk_of(n, reorth);
    return (n + c - 1) / c;
}

size_t lz_workspace_doubles(const ecut_sectors *s, bool reorth, int keep) {
    const int64_t n = s->dim;
    const int64_t nc = n_chunks_of(n, reorth);
    auto al = [](int64_t v) { return (v + 31) & ~(int64_t)31; };
    int64_t d = 0;
    d += reorth ? al(n) * (keep + 1) : al(n) * 3;
    d += al(apply_partial_slots_max(s));
    d += al(nc);
    if (reorth) d += al(nc * keep) + 2 * al(MAX_BASIS);
    d += 32;
    return (size_t)d;
}

void lz_carve(LzSolve &L, const ecut_sectors *s, bool reorth, int keep, double *ws) {
    static std::atomic<uint64_t> next_uid{1};
    L.uid = next_uid++;
    const int64_t n = s->dim;
    const int64_t nc = n_chunks_of(n, reorth);
    auto al = [](int64_t v) { return (v + 31) & ~(int64_t)31; };
    L.chunk = chunk_of(n, reorth);
    L.s = s;
    L.n = n;
    L.reorth = reorth;
    L.keep = keep;
    double *p = ws;
    if (reorth) {
        L.basis = p;
        p += al(n) * (keep + 1);
        // the basis stride is al(n); keep n as the logical length
    } else {
        for (int k = 0; k < 3; ++k) { L.ring[k] = p; p += al(n); }
    }
    L.n_apply = apply_partial_slots(s);
    L.part_apply = p;
    p += al(apply_partial_slots_max(s));
    L.n_chunks = (int32_t)nc;
    L.part_norm = p;
    p += al(nc);
    if (reorth) {
        L.part_cgs = p;
        p += al(nc * keep);
        L.dcoef = p;
        p += al(MAX_BASIS);
        L.dscale = p;
        p += al(MAX_BASIS);
    }
    L.scal = p;
}

static int64_t basis_ld(const LzSolve &L) { return (L.n + 31) & ~(int64_t)31; }

// x/y/z addresses honour the padded basis stride
static double *slot(const LzSolve &L, int k) { return L.basis + (int64_t)k * basis_ld(L); }
static double *xvec(const LzSolve &L) { return L.reorth ? slot(L, L.j) : L.ring[L.j % 3]; }
static double *yvec(const LzSolve &L) { return L.reorth ? slot(L, L.j + 1) : L.ring[(L.j + 1) % 3]; }
static double *zvec(const LzSolve &L) {
    return L.j == 0 ? nullptr : (L.reorth ? slot(L, L.j - 1) : L.ring[(L.j + 2) % 3]);
}

// ---------------------------------------------------------------- descriptor packing
namespace {
struct Pack {
    std::vector<char> buf;
    template <class T>
    size_t put(const std::vector<T> &v) {
        size_t o = (buf.size() + 255) & ~(size_t)255;
        buf.resize(o + v.size() * sizeof(T));
        if (!v.empty()) std::memcpy(buf.data() + o, v.data(), v.size() * sizeof(T));
        return o;
    }
};
}  // namespace

LzPipe::~LzPipe() {
    for (Step &S : steps) {
        if (S.ev) {
            (void)hipEventSynchronize(S.ev);
            (void)hipEventDestroy(S.ev);
        }
        if (S.host) (void)hipHostFree(S.host);
    }
}

// room for n solves in a free step slot (its previous copy has completed)
static ecut_status step_reserve(LzPipe::Step &S, size_t n) {
    if (!S.ev && hipEventCreateWithFlags(&S.ev, hipEventDisableTiming) != hipSuccess)
        return fail(ECUT_EDEVICE, "hipEventCreate (lanczos step)");
    if (n <= S.cap) return ECUT_OK;
    if (S.host) (void)hipHostFree(S.host);
    S.host = S.host_dev = nullptr;
    S.cap = 0;
    size_t c = 64;
    while (c < n) c *= 2;
    // coherent, mapped: the reduction kernel writes alpha, |w|^2 here directly
    if (hipHostMalloc(&S.host, c * 2 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
        return fail(ECUT_ENOMEM, "hipHostMalloc(lanczos scalars)");
    if (hipHostGetDevicePointer((void **)&S.host_dev, S.host, 0) != hipSuccess)
        return fail(ECUT_EDEVICE, "hipHostGetDevicePointer(lanczos scalars)");
    S.cap = c;
    return ECUT_OK;
}

// |v|^2 of each start vector into scal[1], then the first scale 1/|v| and a
// zero previous-vector coefficient, set on the device by the reduction (start mode)
static ecut_status run_start_jobs(std::vector<LzSolve *> &act, const std::vector<double *> &vecs, hipStream_t st,
                                  Staging &stg) {
    std::vector<VecJob> jn, jr;
    std::vector<int32_t> cj, ci;
    for (size_t k = 0; k < act.size(); ++k) {
        LzSolve &L = *act[k];
        VecJob J{};
        J.x = vecs[k];
        J.y = vecs[k];
        J.n = L.n;
        J.partials = L.part_norm;
        J.scalars = L.scal;
        J.coef_idx = 0;
        J.coef_mul = 0.0;
        J.chunk = L.chunk;
        jn.push_back(J);
        for (int32_t c = 0; c < L.n_chunks; ++c) { cj.push_back((int32_t)k); ci.push_back(c); }
        VecJob R{};
        R.partials = L.part_norm;
        R.n_partials = L.n_chunks;
        R.mode = 1;
        R.scalars = L.scal;
        R.out = 1;
        R.next = LzNextJob{L.scal, L.scal + 8, L.reorth ? L.dscale : nullptr, 0, 1};
        jr.push_back(R);
    }
    Pack P;
    size_t o_jn = P.put(jn), o_jr = P.put(jr), o_cj = P.put(cj), o_ci = P.put(ci);
    ecut_status rs = stg.reserve(P.buf.size());
    if (rs != ECUT_OK) return rs;
    rs = stg.wait();
    if (rs != ECUT_OK) return rs;
    std::memcpy(stg.host, P.buf.data(), P.buf.size());
    rs = stg.upload(P.buf.size(), st);
    if (rs != ECUT_OK) return rs;
    char *d = (char *)stg.dev;
    hipError_t e = launch_axpy_norm((const VecJob *)(d + o_jn), (const int32_t *)(d + o_cj), (const int32_t *)(d + o_ci),
                                    (int)cj.size(), st);
    if (e == hipSuccess) e = launch_reduce((const VecJob *)(d + o_jr), (int)jr.size(), st);
    if (e != hipSuccess) return hip_fail(e, "lanczos start");
    return ECUT_OK;
}

ecut_status lz_start(std::vector<LzSolve *> &solves, const std::vector<const double *> &v0, hipStream_t st,
                     Staging &stg, bool host_norm) {
    std::vector<double *> xs;
    std::vector<LzSolve *> act;
    for (size_t k = 0; k < solves.size(); ++k) {
        LzSolve &L = *solves[k];
        L.j = 0;
        L.a.clear();
        L.b.clear();
        L.sc.clear();
        double *x0 = L.reorth ? slot(L, 0) : L.ring[0];
        if (v0[k] && v0[k] != x0) {
            hipError_t e = hipMemcpyAsync(x0, v0[k], sizeof(double) * (size_t)L.n, hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(v0)");
        }
        // alpha must read as zero in the norm pass (coefficient 0 * scal[0])
        hipError_t e = hipMemsetAsync(L.scal, 0, 16 * sizeof(double), st);
        if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync(scal init)");
        xs.push_back(x0);
        act.push_back(&L);
    }
    ecut_status rs = run_start_jobs(act, xs, st, stg);
    if (rs != ECUT_OK || !host_norm) return rs;
    for (LzSolve *L : act) {
        double h[2] = {0.0, 0.0};
        hipError_t e = hipMemcpyAsync(h, L->scal + 8, sizeof(h), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "lanczos start norm");
        L->start_norm2 = h[1];
        const double nrm = std::sqrt(std::max(h[1], 0.0));
        if (!(nrm > 0.0) || !std::isfinite(nrm)) {
            L->done = true;
            L->status = fail(ECUT_EINVAL, "start vector is zero or not finite");
            continue;
        }
        L->sc.push_back(1.0 / nrm);   // the scale set on the device
    }
    return ECUT_OK;
}

ecut_status lz_ritz_vector(LzSolve &L, double *out, hipStream_t st, Staging &stg) {
    if (!L.reorth) return fail(ECUT_EUNSUPPORTED, "Ritz vector needs full reorthogonalisation");
    const int m = (int)L.a.size();
    std::vector<double> e(L.b.begin(), L.b.begin() + (m > 0 ? m - 1 : 0));
    const std::vector<double> ev = tridiag_eigenvalues(L.a, e);
    const std::vector<double> u = tridiag_eigenvector(L.a, e, ev[0]);
    Pack P;
    std::vector<double> scv(L.sc.begin(), L.sc.begin() + m);
    size_t o_c = P.put(u), o_s = P.put(scv);
    ecut_status rs = stg.reserve(P.buf.size());
    if (rs != ECUT_OK) return rs;
    rs = stg.wait();
    if (rs != ECUT_OK) return rs;
    std::memcpy(stg.host, P.buf.data(), P.buf.size());
    rs = stg.upload(P.buf.size(), st);
    if (rs != ECUT_OK) return rs;
    char *d = (char *)stg.dev;
    hipError_t er = launch_multiaxpy(L.basis, basis_ld(L), m, (const double *)(d + o_c), (const double *)(d + o_s), out,
                                     L.n, nullptr, L.n_chunks, 0.0, st);
    if (er != hipSuccess) return hip_fail(er, "Ritz vector");
    return ECUT_OK;
}

bool lz_can_launch(const LzSolve &L) {
    if (L.done) return false;
    if (L.reorth && L.pending > 0) return false;   // a restart may follow each step
    const int limit = L.fixed ? L.max_steps : L.max_steps * (L.max_restarts + 1);
    return L.total + L.pending < limit;
}

// Everything one step launches, with its descriptors packed in one buffer.
namespace {
struct StepPlan {
    std::vector<LzSolve *> act;
    std::vector<ProblemDev> own;              // problems launched on their own kernels
    std::vector<const ecut_sectors *> own_s;
    RowsBatch rows;                           // the others, one row-kernel queue
    bool has_rows = false;
    HubBatch hub;                             // Hubbard problems on the merged two-pass launches
    HubBatchLayout hub_l;
    bool fuse_alpha = false;                  // alpha formed inside the update pass
    Pack P;
    size_t o_rows = 0, o_ja = 0, o_jx = 0, o_jb = 0, o_cj = 0, o_ci = 0, o_n0 = 0, o_n1 = 0;
    int n_ja = 0, n_cj = 0;
    LzSolve *R = nullptr;                     // the one solve with reorthogonalisation, if any
};
}  // namespace

// out2: device room for alpha, |w|^2 of every solve of the step
static void build_plan(const std::vector<LzSolve *> &act, double *out2, StepPlan &pl) {
    pl.act = act;
    // 1. u = s_j H w_j - beta_{j-1} s_{j-1} w_{j-1}, alpha partials; the two
    //    factors are read on the device from scal[LZ_S], scal[LZ_Z]
    std::vector<ProblemDev> rows_probs;
    std::vector<const ecut_sectors *> rows_s;
    std::vector<ItemDev> rows_items;
    std::vector<int32_t> rows_tiles;
    for (LzSolve *L : act) {
        ProblemDev P = L->s->prob;
        P.x = xvec(*L);
        P.y = yvec(*L);
        P.z = zvec(*L);
        P.dscale = L->scal + LZ_S;
        P.partials = L->part_apply;
        if (act.size() > 1 && hub6_batchable(L->s)) {
            hub6_batch_add(pl.hub, L->s, P);
        } else if (own_launch(L->s) || act.size() == 1) {
            pl.own.push_back(P);
            pl.own_s.push_back(L->s);
        } else {
            const int32_t pi = (int32_t)rows_probs.size();
            rows_probs.push_back(P);
            rows_s.push_back(L->s);
            for (const ItemDev &it : L->s->items) rows_items.push_back(ItemDev{pi, it.block, it.row0, it.row1, it.slot, 0});
            rows_tiles.push_back(max_tile_elems(L->s));
        }
    }
    if (!rows_items.empty()) {
        // one work queue over every problem, largest tiles first
        std::stable_sort(rows_items.begin(), rows_items.end(), [&](const ItemDev &a, const ItemDev &b) {
            const int64_t wa = (int64_t)(a.row1 - a.row0) * rows_s[a.prob]->blocks[a.block].d_r;
            const int64_t wb = (int64_t)(b.row1 - b.row0) * rows_s[b.prob]->blocks[b.block].d_r;
            return wa > wb;
        });
        make_rows_batch(rows_probs, rows_items, rows_tiles, pl.rows);
        pl.has_rows = true;
        pl.o_rows = pl.P.put(pl.rows.buf);
    }
    if (!pl.hub.empty()) {
        pl.hub_l = hub6_batch_layout(pl.hub, pl.P.buf.size());
        pl.P.buf.resize(pl.hub_l.bytes);
        hub6_batch_pack(pl.hub, pl.hub_l, pl.P.buf.data());
    }
    // 2.-4. alpha, w = u - alpha v_j with norm partials, beta^2; 5. next factors.
    // When every block of the update pass can afford to re-add the alpha
    // partials (at most 4M reads in all), it does so and alpha needs no launch.
    std::vector<VecJob> ja, jx, jb;
    std::vector<int32_t> cj, ci;
    int64_t alpha_reads = 0;
    for (LzSolve *L : act) alpha_reads += (int64_t)apply_partial_slots(L->s) * L->n_chunks;
    pl.fuse_alpha = alpha_reads <= (int64_t)1 << 22;
    for (size_t k = 0; k < act.size(); ++k) {
        LzSolve &L = *act[k];
        VecJob A{};
        L.n_apply = apply_partial_slots(L.s);   // the tuning may have changed since the workspace was carved
        A.partials = L.part_apply;
        A.n_partials = L.n_apply;
        A.mode = 0;
        A.scalars = L.scal;
        A.out = 0;
        A.dscale = L.scal + LZ_S;
        ja.push_back(A);
        VecJob X{};
        X.x = xvec(L);
        X.y = yvec(L);
        X.n = L.n;
        X.partials = L.part_norm;
        X.scalars = L.scal;
        X.coef_idx = 0;
        X.dscale = L.scal + LZ_S;
        X.chunk = L.chunk;
        if (pl.fuse_alpha) {
            X.a_partials = L.part_apply;
            X.a_n = L.n_apply;
        }
        jx.push_back(X);
        for (int32_t c = 0; c < L.n_chunks; ++c) { cj.push_back((int32_t)k); ci.push_back(c); }
        VecJob B{};
        B.partials = L.part_norm;
        B.n_partials = L.n_chunks;
        B.mode = 1;
        B.scalars = L.scal;
        B.out = 1;
        B.next = LzNextJob{L.scal, out2 + 2 * k, L.reorth ? L.dscale : nullptr, L.j + 1, 0};
        jb.push_back(B);
    }
    pl.o_ja = pl.P.put(ja);
    pl.o_jx = pl.P.put(jx);
    pl.o_jb = pl.P.put(jb);
    pl.o_cj = pl.P.put(cj);
    pl.o_ci = pl.P.put(ci);
    pl.n_ja = (int)ja.size();
    pl.n_cj = (int)cj.size();
    pl.R = (act.size() == 1 && act[0]->reorth) ? act[0] : nullptr;
    if (pl.R) {
        // squared norm of w before (scal[2]) and after (scal[3]) the first projection
        std::vector<VecJob> n0(1), n1(1);
        n0[0].partials = pl.R->part_norm;
        n0[0].n_partials = pl.R->n_chunks;
        n0[0].mode = 1;
        n0[0].scalars = pl.R->scal;
        n0[0].out = 2;
        n1[0] = n0[0];
        n1[0].out = 3;
        pl.o_n0 = pl.P.put(n0);
        pl.o_n1 = pl.P.put(n1);
    }
}

// launches of a step; dev: a device copy of pl.P.buf
static ecut_status enqueue_plan(const StepPlan &pl, const void *dev, hipStream_t st) {
    for (size_t k = 0; k < pl.own.size(); ++k) {
        ecut_status rs = launch_apply(pl.own_s[k], pl.own[k], st);
        if (rs != ECUT_OK) return rs;
    }
    const char *d = (const char *)dev;
    hipError_t e = hipSuccess;
    if (pl.has_rows) e = launch_rows_batch(pl.rows, d + pl.o_rows, st);
    if (e == hipSuccess) e = hub6_batch_launch(pl.hub, pl.hub_l, d, st);
    if (e != hipSuccess) return hip_fail(e, "kernel launch (batched apply_H)");
    if (!pl.fuse_alpha) e = launch_reduce((const VecJob *)(d + pl.o_ja), pl.n_ja, st);
    if (e == hipSuccess)
        e = launch_axpy_norm((const VecJob *)(d + pl.o_jx), (const int32_t *)(d + pl.o_cj), (const int32_t *)(d + pl.o_ci),
                             pl.n_cj, st);
    if (e != hipSuccess) return hip_fail(e, "lanczos update");
    if (LzSolve *R = pl.R) {
        // classical Gram-Schmidt against w_0..w_j (v_k = s_k w_k, the scales
        // kept on the device by the reductions); the second pass runs only when the
        // first one removed more than half of the squared norm (decided on
        // the device).  Every pass leaves the norm partials of its result in
        // part_norm, so beta^2 below is the norm of the vector actually kept.
        const int nv = R->j + 1;
        if (nv > MAX_BASIS) return fail(ECUT_EUNSUPPORTED, "too many basis vectors");
        e = launch_reduce((const VecJob *)(d + pl.o_n0), 1, st);
        const double *gate = R->scal + 4;
        for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
            const double *g = pass == 1 ? gate : nullptr;
            e = launch_multidot(R->basis, basis_ld(*R), nv, yvec(*R), R->n, R->part_cgs, R->n_chunks, st, g);
            if (e == hipSuccess) e = launch_multidot_reduce(R->part_cgs, R->n_chunks, nv, R->dscale, R->dcoef, st, g);
            if (e == hipSuccess)
                e = launch_multiaxpy(R->basis, basis_ld(*R), nv, R->dcoef, R->dscale, yvec(*R), R->n, R->part_norm,
                                     R->n_chunks, 1.0, st, g);
            if (e == hipSuccess && pass == 0) e = launch_reduce((const VecJob *)(d + pl.o_n1), 1, st);
            if (e == hipSuccess && pass == 0) e = launch_dgks_gate(R->scal, st);
        }
        if (e != hipSuccess) return hip_fail(e, "reorthogonalisation");
    }
    e = launch_reduce((const VecJob *)(d + pl.o_jb), (int)pl.act.size(), st);   // and the next factors
    if (e != hipSuccess) return hip_fail(e, "lanczos beta");
    return ECUT_OK;
}

LzGraph::~LzGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (dev) (void)hipFreeAsync(dev, st);
    if (dev_out) (void)hipFreeAsync(dev_out, st);
}

std::mutex &lz_capture_mutex() {
    static std::mutex m;
    return m;
}

// capture one step of act (its current ring phases) as a graph
static ecut_status capture_step(const std::vector<LzSolve *> &act, hipStream_t st, std::shared_ptr<LzGraph> &out) {
    auto g = std::make_shared<LzGraph>();
    g->st = st;
    hipError_t e = hipMallocAsync((void **)&g->dev_out, 2 * sizeof(double) * act.size(), st);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync(graph scalars)");
    StepPlan pl;
    build_plan(act, g->dev_out, pl);
    e = hipMallocAsync(&g->dev, pl.P.buf.size(), st);
    if (e == hipSuccess) e = hipMemcpyAsync(g->dev, pl.P.buf.data(), pl.P.buf.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // the pageable source is released on return
    if (e != hipSuccess) return hip_fail(e, "graph descriptors");
    ecut_status rs;
    hipGraph_t graph = nullptr;
    {
        std::lock_guard<std::mutex> cg(lz_capture_mutex());
        e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        rs = enqueue_plan(pl, g->dev, st);
        e = hipStreamEndCapture(st, &graph);
    }
    if (rs != ECUT_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rs;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    out = g;
    return ECUT_OK;
}

ecut_status lz_launch(std::vector<LzSolve *> &solves, LzPipe &pipe, hipStream_t st, Staging &stg) {
    if (pipe.n >= LzPipe::DEPTH) return fail(ECUT_EINVAL, "Lanczos pipe full");
    std::vector<LzSolve *> act;
    for (LzSolve *L : solves)
        if (lz_can_launch(*L)) act.push_back(L);
    if (act.empty()) return ECUT_OK;
    LzPipe::Step &S = pipe.steps[(pipe.head + pipe.n) % LzPipe::DEPTH];
    ecut_status rs = step_reserve(S, act.size());
    if (rs != ECUT_OK) return rs;
    // graph replay: three-term solves past their first step, launched by the
    // previous step too (a new set of solves drops the captured graphs)
    std::vector<uint64_t> who, key;
    bool graph = pipe.use_graph && st != nullptr;
    for (LzSolve *L : act) {
        who.push_back(L->uid);
        key.push_back(L->uid);
        key.push_back((uint64_t)(L->j % 3));
        graph = graph && !L->reorth && L->j >= 1;
    }
    if (who != pipe.last) {
        pipe.graphs.clear();   // graphs of a launch still in flight live on in its step
        pipe.last = who;
        pipe.same = 0;
    } else {
        ++pipe.same;
    }
    graph = graph && pipe.same >= LzPipe::GRAPH_AFTER;
    hipError_t e;
    if (graph) {
        std::shared_ptr<LzGraph> &g = pipe.graphs[key];
        if (!g) {
            rs = capture_step(act, st, g);
            if (rs != ECUT_OK) return rs;
            ++pipe.graph_captures;
        }
        ++pipe.graph_replays;
        e = hipGraphLaunch(g->exec, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(S.host, g->dev_out, 2 * sizeof(double) * act.size(), hipMemcpyDeviceToHost, st);
        S.graph = g;
    } else {
        StepPlan pl;
        build_plan(act, S.host_dev, pl);   // alpha, |w|^2 go straight to pinned host memory
        rs = stg.reserve(pl.P.buf.size());
        if (rs != ECUT_OK) return rs;
        rs = stg.wait();
        if (rs != ECUT_OK) return rs;
        std::memcpy(stg.host, pl.P.buf.data(), pl.P.buf.size());
        rs = stg.upload(pl.P.buf.size(), st);
        if (rs != ECUT_OK) return rs;
        rs = enqueue_plan(pl, stg.dev, st);
        if (rs != ECUT_OK) return rs;
        e = hipSuccess;
        S.graph.reset();
    }
    if (e == hipSuccess) e = hipEventRecord(S.ev, st);
    if (e != hipSuccess) return hip_fail(e, "lanczos step");
    S.solves = act;
    for (LzSolve *L : act) {
        ++L->pending;
        ++L->j;
    }
    ++pipe.n;
    return ECUT_OK;
}

ecut_status lz_finish(LzPipe &pipe, hipStream_t st, Staging &stg) {
    if (pipe.n == 0) return ECUT_OK;
    LzPipe::Step &S = pipe.steps[pipe.head];
    hipError_t e = hipEventSynchronize(S.ev);
    pipe.head = (pipe.head + 1) % LzPipe::DEPTH;
    --pipe.n;
    std::vector<LzSolve *> act;
    act.swap(S.solves);
    S.graph.reset();
    for (LzSolve *L : act) --L->pending;
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize (lanczos step)");
    // host: tridiagonal eigenproblem and convergence
    for (size_t k = 0; k < act.size(); ++k) {
        LzSolve *L = act[k];
        if (L->done) continue;   // a step launched before the solve was seen to stop
        const double alpha = S.host[2 * k];
        const double beta = std::sqrt(std::max(S.host[2 * k + 1], 0.0));
        if (!std::isfinite(alpha) || !std::isfinite(beta)) {
            L->done = true;
            L->status = fail(ECUT_EDEVICE, "non-finite Lanczos coefficient");
            continue;
        }
        L->a.push_back(alpha);
        L->b.push_back(beta);
        ++L->total;
        const int m = (int)L->a.size();
        std::vector<double> eo(L->b.begin(), L->b.begin() + (m - 1));
        // O(m) per step: bisection from the previous Ritz value (an upper
        // bound by interlacing), inverse iteration for the last component
        const double lowest = tridiag_lowest(L->a, eo, m > 1 ? L->energy : NAN, L->energy - L->e_prev);
        const std::vector<double> u = tridiag_eigenvector(L->a, eo, lowest);
        L->e_prev = m > 1 ? L->energy : lowest;
        L->energy = lowest;
        L->residual = beta * std::fabs(u[m - 1]);
        const bool breakdown = beta <= 1e-14 * std::max(std::fabs(alpha), 1e-300);
        const bool conv = (L->residual <= 1e-2 * std::sqrt(L->tol) && m > 1 && std::fabs(L->energy - L->e_prev) <= L->tol);
        if (L->fixed) {
            if (L->total >= L->max_steps || breakdown) L->done = true;
        } else if (conv || breakdown) {
            L->done = true;
        } else if (L->total >= L->max_steps * (L->max_restarts + 1)) {
            L->done = true;
            L->status = ECUT_ENOTCONV;
        }
        if (L->done) continue;
        if (L->reorth && m >= L->keep) {
            // explicit restart from the current Ritz vector
            if (L->restarts >= L->max_restarts) {
                L->done = true;
                L->status = ECUT_ENOTCONV;
                continue;
            }
            ecut_status r2 = lz_ritz_vector(*L, slot(*L, 0), st, stg);
            if (r2 != ECUT_OK) return r2;
            ++L->restarts;
            std::vector<LzSolve *> one{L};
            std::vector<const double *> v0{slot(*L, 0)};
            r2 = lz_start(one, v0, st, stg, true);
            if (r2 != ECUT_OK) return r2;
            continue;
        }
        if (L->reorth) L->sc.push_back(1.0 / beta);   // the scale set on the device
    }
    return ECUT_OK;
}

ecut_status lz_step(std::vector<LzSolve *> &solves, LzPipe &pipe, hipStream_t st, Staging &stg) {
    ecut_status rs = lz_launch(solves, pipe, st, stg);
    while (rs == ECUT_OK && pipe.n > 0) rs = lz_finish(pipe, st, stg);
    return rs;
}

// Final energy: all eigenvalues of T by implicit QL; the per-step bisection
// value must agree with it.
double final_energy(const LzSolve &L) {
    if (L.a.empty()) return L.energy;
    std::vector<double> eo(L.b.begin(), L.b.begin() + (L.a.size() - 1));
    const double ql = tridiag_eigenvalues(L.a, eo)[0];
    return std::fabs(ql - L.energy) <= 1e-9 * (std::fabs(ql) + 1.0) ? ql : L.energy;
}

// One solve on the calling thread: carve the workspace, start, and run the
// steps (two in flight without reorthogonalisation) until the solve stops.
static ecut_status solve_one(const ecut_sectors *s, const double *v0_d, const ecut_lanczos_opts *opts,
                             double *basis_d, hipStream_t &st, Staging &stg, LzSolve &L) {
    if (opts->use_graph && !st) {
        // graphs are captured on a stream of our own, ordered after the
        // caller's work on the null stream; the call is synchronous anyway
        static thread_local hipStream_t priv = nullptr;
        static thread_local hipEvent_t after = nullptr;
        hipError_t e = hipSuccess;
        if (!priv) e = hipStreamCreateWithFlags(&priv, hipStreamNonBlocking);
        if (e == hipSuccess && !after) e = hipEventCreateWithFlags(&after, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(after, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(priv, after, 0);
        if (e != hipSuccess) return hip_fail(e, "lanczos stream");
        st = priv;
    }
    lz_carve(L, s, opts->reorth != 0, opts->reorth ? opts->max_steps : 0, basis_d);
    L.max_steps = opts->max_steps;
    L.max_restarts = opts->max_restarts;
    L.fixed = opts->fixed_steps != 0;
    L.tol = opts->tol;
    std::vector<LzSolve *> v{&L};
    std::vector<const double *> v0{v0_d};
    ecut_status rs = lz_start(v, v0, st, stg, true);
    if (rs != ECUT_OK) return rs;
    if (L.done) return L.status;
    // three-term solves keep two steps in flight: the host processes step j
    // while the device runs step j + 1 (its factors are set on the device),
    // so a converged solve runs one extra step whose result is dropped
    LzPipe pipe;
    pipe.use_graph = opts->use_graph != 0;
    while (!L.done || pipe.n > 0) {
        if (!L.done && pipe.n < LzPipe::DEPTH && lz_can_launch(L)) {
            rs = lz_launch(v, pipe, st, stg);
        } else if (pipe.n > 0) {
            rs = lz_finish(pipe, st, stg);
        } else {
            L.done = true;   // no step left to launch: the budget ends the solve
            L.status = L.fixed ? ECUT_OK : ECUT_ENOTCONV;
        }
        if (rs != ECUT_OK) {
            (void)hipStreamSynchronize(st);
            return rs;
        }
    }
    if (L.status != ECUT_OK && L.status != ECUT_ENOTCONV) return L.status;
    return ECUT_OK;
}

}  // namespace ecut

using namespace ecut;

extern "C" {

size_t ecut_lanczos_workspace(const ecut_sectors *s, const ecut_lanczos_opts *opts) {
    if (!s || !opts) return 0;
    const bool re = opts->reorth != 0;
    return lz_workspace_doubles(s, re, re ? opts->max_steps : 0);
}

ecut_status ecut_lanczos_ground_state(const ecut_sectors *s, const double *v0_d, const ecut_lanczos_opts *opts,
                                      double *energy, double *gs_d, ecut_lanczos_stats *stats, double *basis_d,
                                      void *stream) {
    if (!s || !opts || !energy || !v0_d || !basis_d) return fail(ECUT_EINVAL, "null argument");
    if (!s->on_device) return fail(ECUT_EINVAL, "handle was built with ECUT_BUILD_HOST_ONLY");
    if (opts->max_steps < 1) return fail(ECUT_EINVAL, "max_steps must be >= 1");
    if (opts->max_restarts < 0) return fail(ECUT_EINVAL, "max_restarts must be >= 0");
    if (opts->reorth && opts->max_steps + 1 > MAX_BASIS) return fail(ECUT_EUNSUPPORTED, "max_steps too large for reorth");
    if (!opts->fixed_steps && !(opts->tol > 0.0)) return fail(ECUT_EINVAL, "tol must be > 0");
    if (gs_d && !opts->reorth) return fail(ECUT_EUNSUPPORTED, "gs_d needs reorth = 1");
    if (opts->max_restarts > 0 && !opts->reorth) return fail(ECUT_EUNSUPPORTED, "restarts need reorth = 1");
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    static thread_local Staging stg;
    LzSolve L;
    ecut_status rs = solve_one(s, v0_d, opts, basis_d, st, stg, L);
    if (rs != ECUT_OK) return rs;
    *energy = final_energy(L);
    if (gs_d) {
        rs = lz_ritz_vector(L, gs_d, st, stg);
        if (rs != ECUT_OK) return rs;
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize (ground state)");
    }
    if (stats) {
        stats->steps = L.total;
        stats->restarts = L.restarts;
        stats->converged = L.status == ECUT_OK && !L.fixed ? 1 : 0;
        stats->residual = L.residual;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (L.status == ECUT_ENOTCONV) return fail(ECUT_ENOTCONV, "Lanczos did not reach tol");
    return ECUT_OK;
}

ecut_status ecut_lanczos_tridiag(const ecut_sectors *s, const double *v0_d, int32_t n_steps, double *alpha,
                                 double *beta, int32_t *n_out, double *v0_norm2, double *basis_d, void *stream) {
    if (!s || !v0_d || !alpha || !beta || !n_out || !basis_d) return fail(ECUT_EINVAL, "null argument");
    if (!s->on_device) return fail(ECUT_EINVAL, "handle was built with ECUT_BUILD_HOST_ONLY");
    if (n_steps < 1) return fail(ECUT_EINVAL, "n_steps must be >= 1");
    ecut_lanczos_opts o{};
    o.max_steps = n_steps;
    o.fixed_steps = 1;
    hipStream_t st = (hipStream_t)stream;
    static thread_local Staging stg;
    LzSolve L;
    *n_out = 0;
    ecut_status rs = solve_one(s, v0_d, &o, basis_d, st, stg, L);
    if (v0_norm2) *v0_norm2 = L.start_norm2;
    if (rs != ECUT_OK) return rs;
    const int m = (int)L.a.size();
    for (int j = 0; j < m; ++j) {
        alpha[j] = L.a[j];
        beta[j] = L.b[j];
    }
    *n_out = m;
    return ECUT_OK;
}

ecut_status ecut_continued_fraction(const double *alpha, const double *beta, int32_t n, double weight, double e0,
                                    int32_t dagger, const double *omega, int32_t n_omega, double eta, double *g_re,
                                    double *g_im) {
    if (!alpha || !beta || !omega || !g_re || !g_im || n < 1 || n_omega < 0) return fail(ECUT_EINVAL, "bad argument");
    const double sgn = dagger ? 1.0 : -1.0;
    for (int32_t k = 0; k < n_omega; ++k) {
        const std::complex<double> z(omega[k] + (dagger ? e0 : -e0), eta);
        std::complex<double> g(0.0, 0.0);
        for (int32_t j = n - 1; j >= 0; --j) {
            const std::complex<double> tail = j + 1 < n ? beta[j] * beta[j] * g : std::complex<double>(0.0, 0.0);
            g = 1.0 / (z - sgn * alpha[j] - tail);
        }
        g *= weight;
        g_re[k] = g.real();
        g_im[k] = g.imag();
    }
    return ECUT_OK;
}

}  // extern "C"

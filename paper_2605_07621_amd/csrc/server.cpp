// Continuous-batching ground-state server.
//
// A worker thread owns one HIP stream and a device arena of hbm_budget
// bytes.  Each step it
//   1. admits queued requests (FIFO, arrival time reached) while a slot is
//      free and the request's Lanczos workspace fits the free arena;
//   2. launches one Lanczos step of every admitted solve: one batched H*psi
//      launch over the sector work queue of all generic-kernel problems (plus
//      the Hubbard up/down kernel per Hubbard problem), one batched alpha
//      reduction, one batched update+norm pass, one batched beta reduction
//      and the next step's factors, all on the device, then one copy of all
//      alpha/beta values to pinned host memory;
//   3. with two steps in flight, waits for the older one and checks its
//      solves (convergence, breakdown) while the device runs the newer one;
//   4. retires finished solves once no step of theirs is in flight, freeing
//      their arena space and slot.
// With max_active = 1 the same loop is the sequential baseline: one request
// at a time on the same engine.
// A two-lane server (large_dim > 0) runs this loop on two workers, each with
// its own stream: lane 1 admits the requests of at least large_dim
// amplitudes, lane 0 the others, both from the one arrival-ordered queue and
// the one arena.  Lane 1 runs one request at a time, with the tuning for a
// problem alone, so a large request never shares its steps; lane 0 batches
// the rest, and the two lanes' kernels overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ecut_internal.h"
#include "kernels.h"
#include "lanczos.h"
#include "runtime.h"

namespace ecut {
namespace {

// First-fit allocator over [0, size) with coalescing, 256-byte granules.
struct ArenaAlloc {
    size_t size = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    void init(size_t n) {
        size = n & ~(size_t)255;
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t &off) {
        n = (n + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                off = it->first;
                const size_t rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = (n + 255) & ~(size_t)255;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t free_bytes() const {
        size_t s = 0;
        for (auto &kv : free_) s += kv.second;
        return s;
    }
};

struct Request {
    uint64_t id = 0;
    ecut_model_desc model{};
    ecut_cut_desc cut{};
    ecut_qnum q{};
    uint64_t seed = 0;
    double not_before = 0.0, t_submit = 0.0;
    std::vector<int32_t> bi, bj;
    std::vector<double> jxy, jz, t, u, v;
    // sectors built ahead of admission by the helper thread (or kept while
    // the request waits for memory); state 0 not built, 1 building, 2 built
    ecut_sectors *built = nullptr;
    int state = 0;
    ecut_status build_status = ECUT_OK;
    int lane = 0;   // the worker that admits it (1: a large request of a two-lane server)
    ~Request() {
        if (built) ecut_sectors_free(built);
    }
    void own(const ecut_model_desc &m) {
        model = m;
        bi.assign(m.bond_i, m.bond_i + m.n_bonds);
        bj.assign(m.bond_j, m.bond_j + m.n_bonds);
        if (m.jxy) jxy.assign(m.jxy, m.jxy + m.n_bonds);
        if (m.jz) jz.assign(m.jz, m.jz + m.n_bonds);
        if (m.t) t.assign(m.t, m.t + m.n_bonds);
        if (m.u) u.assign(m.u, m.u + m.n_sites);
        if (m.v) v.assign(m.v, m.v + m.n_bonds);
        model.bond_i = bi.data();
        model.bond_j = bj.data();
        model.jxy = m.jxy ? jxy.data() : nullptr;
        model.jz = m.jz ? jz.data() : nullptr;
        model.t = m.t ? t.data() : nullptr;
        model.u = m.u ? u.data() : nullptr;
        model.v = m.v ? v.data() : nullptr;
    }
};

struct Active {
    std::unique_ptr<Request> req;
    ecut_sectors *s = nullptr;
    LzSolve L;
    size_t off = 0, bytes = 0;
    double t_admit = 0.0;
};

}  // namespace
}  // namespace ecut

using namespace ecut;

// One worker with its own stream and staging buffers.  A two-lane server
// runs large requests on lane 1 and the others on lane 0; each lane batches
// its own solves, and the two streams' kernels overlap on the device.
struct ServerLane {
    hipStream_t stream = nullptr;
    Staging stg;
    std::thread worker;
};

struct ecut_server {
    size_t budget = 0;
    ecut_server_opts opts{};
    int device = 0;
    void *arena = nullptr;
    ArenaAlloc alloc;   // shared by the lanes, guarded by mu
    ServerLane lanes[2];
    int n_lanes = 1;
    // lane k's head is built and has a free slot but waits for arena space;
    // the other lane then admits nothing that arrived after it (guarded by mu)
    bool mem_wait[2] = {false, false};
    std::thread helper;
    std::mutex mu;
    std::condition_variable cv, cv_done, cv_help;
    std::vector<ecut_sectors *> graveyard;   // retired handles, freed by the helper
    std::deque<std::unique_ptr<Request>> queue;
    std::vector<ecut_result> finished;
    uint64_t next_id = 1;
    uint64_t n_submitted = 0, n_finished = 0;
    bool stop = false;
    std::chrono::steady_clock::time_point t0;
    ecut_status worker_status = ECUT_OK;
    std::string worker_msg;   // the worker's error message (error messages are per thread)

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
    // the oldest queued request of a lane (mu held), or the end of the queue
    std::deque<std::unique_ptr<Request>>::iterator head(int lane) {
        return std::find_if(queue.begin(), queue.end(), [lane](const std::unique_ptr<Request> &r) { return r->lane == lane; });
    }
    void run(int lane);
    void help();
};

static size_t footprint(const ecut_sectors *s) { return lz_workspace_doubles(s, false, 0) * sizeof(double); }

// Amplitudes of a request's sector (any cut gives the same count): C(n, N_up)
// for spins, C(n, N_up) C(n, N_dn) for Hubbard; 0 for numbers out of range.
static double sector_states(const ecut_model_desc &m, ecut_qnum q) {
    auto c = [](int n, int k) {
        if (k < 0 || k > n) return 0.0;
        double r = 1.0;
        for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
        return r;
    };
    return m.kind == ECUT_HUBBARD ? c(m.n_sites, q.n_up) * c(m.n_sites, q.n_dn) : c(m.n_sites, q.n_up);
}

// Launch tuning of each problem shape, measured once per process (on the
// first request of the shape, x = its start vector, y = a ring vector the
// solve overwrites later) and reused for every later request of the shape.
static std::mutex g_tune_mu;
// Hubbard problems up to this many amplitudes (chains of up to 10 sites at
// half filling) share the merged two-pass launches of a step
static constexpr int64_t SMALL_HUB_DIM = (int64_t)1 << 18;
static constexpr int64_t SMALL_SPIN_DIM = (int64_t)1 << 20;
static std::map<std::string, ecut_tuning> g_tunings;

// merged: the tuning of a server that runs several solves per step (small
// problems then prefer the kernels whose launches merge across problems);
// else the autotuner's pick for the problem alone.  Kept per shape and mode
// for the life of the process.
static ecut_status tune_once(ecut_sectors *s, const double *x, double *y, hipStream_t st, bool merged) {
    const std::string key = tune_shape_key(s) + (merged ? "|merged" : "|alone");
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tunings.find(key);
        if (it != g_tunings.end() && ecut_set_tuning(s, &it->second) == ECUT_OK) return ECUT_OK;
    }
    ecut_tuning best{};
    ecut_status rs;
    if (merged && s->kernel == 1 && s->hub6_ok && s->dim <= SMALL_HUB_DIM && s->h6_maxq <= HUBD_BATCH_SLOTS) {
        // small Hubbard problems take the two-pass kernels, so that every
        // step runs all of them in one merged launch per pass
        best = ecut_tuning{0, 8, 1, 6, 2};
        rs = ecut_set_tuning(s, &best);
    } else {
        rs = ecut_autotune(s, x, y, st, &best);
        if (rs == ECUT_OK && merged && s->spin_ok && s->dim <= SMALL_SPIN_DIM && best.variant != 0) {
            // small spin problems keep the one-pass kernel, whose work items
            // join every other spin problem's in one merged launch per step
            best = ecut_tuning{0, 0, 0, 0, 0};
            rs = ecut_set_tuning(s, &best);
        }
    }
    if (rs != ECUT_OK) return rs;
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tunings.emplace(key, best);
    return ECUT_OK;
}

// Helper thread: builds the sectors of arrived requests near the head of the
// queue (at most LOOKAHEAD of them) before the worker admits them, and frees
// the handles of retired solves, so that neither the host work of a build
// nor the device wait inside hipFree sits between two batched steps.
static constexpr int LOOKAHEAD = 16;

void ecut_server::help() {
    const hipError_t dev_err = hipSetDevice(device);   // a failure fails every build
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        if (!graveyard.empty()) {
            std::vector<ecut_sectors *> g;
            g.swap(graveyard);
            lk.unlock();
            {
                std::lock_guard<std::mutex> cg(lz_capture_mutex());
                for (ecut_sectors *s : g) ecut_sectors_free(s);
            }
            lk.lock();
            continue;
        }
        if (stop) break;
        Request *R = nullptr;
        int k = 0;
        const double t = now();
        for (auto &q : queue) {
            if (k++ >= LOOKAHEAD || q->not_before > t) break;   // never ahead of arrival
            if (q->state == 0) {
                R = q.get();
                break;
            }
        }
        if (!R) {
            cv_help.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        R->state = 1;
        lk.unlock();
        ecut_sectors *s = nullptr;
        ecut_status st;
        {
            std::lock_guard<std::mutex> cg(lz_capture_mutex());
            st = dev_err != hipSuccess ? hip_fail(dev_err, "hipSetDevice (server helper)")
                                       : ecut_build_sectors(&R->model, &R->cut, R->q, 0, &s);
        }
        lk.lock();
        R->built = s;
        R->build_status = st;
        R->state = 2;
        cv.notify_all();
    }
}

void ecut_server::run(int lane) {
    hipStream_t stream = lanes[lane].stream;
    Staging &stg = lanes[lane].stg;
    const hipError_t dev_err = hipSetDevice(device);
    if (dev_err != hipSuccess) {   // nothing can run: drain and poll report it
        const ecut_status st = hip_fail(dev_err, "hipSetDevice (server worker)");
        std::lock_guard<std::mutex> g(mu);
        worker_status = st;
        worker_msg = ecut_last_error();
        cv_done.notify_all();
        return;
    }
    std::vector<std::unique_ptr<Active>> active;
    LzPipe pipe;   // batched steps in flight (two: the host processes one while the device runs the next)
    pipe.use_graph = opts.use_graph != 0;
    // the large lane runs its requests one at a time: they are bandwidth-bound,
    // so sharing steps among them would only stretch each one's latency
    const int max_active = lane == 1 ? 1 : opts.max_active > 0 ? opts.max_active : 1 << 30;
    while (true) {
        // ---- admission
        std::vector<Active *> fresh;
        {
            std::unique_lock<std::mutex> lk(mu);
            while (!stop && active.empty()) {
                const auto h = head(lane);
                if (h != queue.end()) {
                    const double wait = (*h)->not_before - now();
                    if (wait <= 0 && (*h)->state == 2) break;
                    // not arrived yet, or the helper is still building it
                    cv.wait_for(lk, std::chrono::duration<double>(wait > 0 ? std::min(wait, 0.05) : 0.05));
                } else {
                    cv.wait_for(lk, std::chrono::milliseconds(50));
                }
            }
            if (stop && active.empty()) break;
            // strict FIFO within the lane; the arena allocator is guarded by mu.
            // Across lanes, no request takes memory ahead of an earlier one of
            // the other lane that waits for it.
            for (auto h = head(lane); h != queue.end() && (int)active.size() < max_active &&
                                      (*h)->not_before <= now() && (*h)->state == 2;
                 h = head(lane)) {
                if (n_lanes > 1 && mem_wait[1 - lane]) {
                    const auto o = head(1 - lane);
                    if (o != queue.end() && o < h) break;
                }
                Request &R = **h;
                ecut_sectors *s = R.built;
                R.built = nullptr;
                ecut_status st = R.build_status;
                size_t off = 0, bytes = 0;
                bool fits = false;
                if (st == ECUT_OK) {
                    bytes = footprint(s);
                    fits = alloc.alloc(bytes, off);
                    if (!fits && bytes > alloc.size) st = fail(ECUT_ENOMEM, "request larger than the server budget");
                }
                mem_wait[lane] = st == ECUT_OK && !fits;
                if (st != ECUT_OK) {
                    ecut_result r{};
                    r.req_id = R.id;
                    r.status = st;
                    r.t_submit = R.t_submit;
                    r.t_admit = r.t_done = now();
                    finished.push_back(r);
                    ++n_finished;
                    queue.erase(h);
                    if (s) ecut_sectors_free(s);
                    cv_done.notify_all();
                    continue;
                }
                if (!fits) {
                    // wait for memory: strict FIFO, the lane's head is never overtaken
                    R.built = s;
                    break;
                }
                cv_help.notify_one();   // the look-ahead window moves on
                auto A = std::make_unique<Active>();
                A->req = std::move(*h);
                queue.erase(h);
                A->s = s;
                A->off = off;
                A->bytes = bytes;
                A->t_admit = now();
                lz_carve(A->L, s, false, 0, (double *)((char *)arena + off));
                A->L.max_steps = opts.max_steps;
                A->L.max_restarts = 0;
                A->L.tol = opts.tol;
                fresh.push_back(A.get());
                active.push_back(std::move(A));
            }
            // an idle lane whose head waits for arena space the other lane
            // holds, or stands behind an earlier request of the other lane that
            // waits for it: sleep until a retirement (or a short timeout)
            if (active.empty() && !stop) cv.wait_for(lk, std::chrono::milliseconds(2));
        }
        ecut_status st = ECUT_OK;
        if (!fresh.empty()) {
            std::vector<LzSolve *> ls;
            std::vector<const double *> v0;
            for (Active *A : fresh) {
                hipError_t e = launch_fill_normal(A->L.ring[0], A->L.n, A->req->seed, stream);
                if (e != hipSuccess) st = hip_fail(e, "seeded start vector");
                if (st == ECUT_OK && opts.autotune)
                    st = tune_once(A->s, A->L.ring[0], A->L.ring[1], stream, max_active > 1);
                ls.push_back(&A->L);
                v0.push_back(A->L.ring[0]);
            }
            if (st == ECUT_OK) st = lz_start(ls, v0, stream, stg, false);
        }
        // ---- one batched step launched, the oldest one in flight processed
        if (st == ECUT_OK && !active.empty()) {
            std::vector<LzSolve *> ls;
            bool any = false;
            for (auto &A : active) {
                ls.push_back(&A->L);
                any = any || lz_can_launch(A->L);
            }
            const int before = pipe.n;
            if (any && pipe.n < LzPipe::DEPTH) st = lz_launch(ls, pipe, stream, stg);
            if (st == ECUT_OK && (pipe.n == LzPipe::DEPTH || (pipe.n == before && pipe.n > 0))) st = lz_finish(pipe, stream, stg);
            if (st == ECUT_OK && pipe.n == 0)
                for (auto &A : active)
                    if (!A->L.done && !lz_can_launch(A->L)) A->L.done = true, A->L.status = ECUT_ENOTCONV;
        }
        if (st != ECUT_OK) {
            (void)hipStreamSynchronize(stream);
            while (pipe.n > 0) (void)lz_finish(pipe, stream, stg);
            std::lock_guard<std::mutex> g(mu);
            worker_status = st;
            worker_msg = ecut_last_error();
            for (auto &A : active) A->L.done = true, A->L.status = st, A->L.pending = 0;
        }
        // ---- retire
        std::vector<ecut_result> out;
        std::vector<ecut_sectors *> retired;
        std::vector<std::pair<size_t, size_t>> spans;   // arena space of the retired solves
        for (auto it = active.begin(); it != active.end();) {
            Active &A = **it;
            if (!A.L.done || A.L.pending > 0) { ++it; continue; }   // retire once no step of it is in flight
            ecut_result r{};
            r.req_id = A.req->id;
            r.status = A.L.status;
            r.steps = A.L.total;
            r.energy = final_energy(A.L);
            r.residual = A.L.residual;
            r.t_submit = A.req->t_submit;
            r.t_admit = A.t_admit;
            r.t_done = now();
            out.push_back(r);
            spans.emplace_back(A.off, A.bytes);
            retired.push_back(A.s);   // freed by the helper: hipFree waits for the device
            it = active.erase(it);
        }
        if (!retired.empty()) {
            std::lock_guard<std::mutex> g(mu);
            for (auto &sp : spans) alloc.release(sp.first, sp.second);
            graveyard.insert(graveyard.end(), retired.begin(), retired.end());
            retired.clear();
            cv_help.notify_one();
            cv.notify_all();   // the other lane may be waiting for memory
        }
        if (!out.empty()) {
            std::lock_guard<std::mutex> g(mu);
            for (auto &r : out) finished.push_back(r);
            n_finished += out.size();
            cv_done.notify_all();
        }
    }
}

extern "C" {

ecut_status ecut_server_create(size_t hbm_budget, const ecut_server_opts *opts, ecut_server **out) {
    if (!out || !opts) return fail(ECUT_EINVAL, "null argument");
    *out = nullptr;
    if (hbm_budget < 4096) return fail(ECUT_EINVAL, "budget too small");
    if (opts->max_steps < 2 || !(opts->tol > 0.0) || opts->large_dim < 0) return fail(ECUT_EINVAL, "bad server options");
    if (opts->large_dim > 0 && opts->use_graph && !opts->sequential)
        return fail(ECUT_EINVAL, "a two-lane server does not replay graphs (large_dim > 0 with use_graph)");
    auto *S = new (std::nothrow) ecut_server();
    if (!S) return fail(ECUT_ENOMEM, "host allocation");
    S->budget = hbm_budget;
    S->opts = *opts;
    if (S->opts.sequential) S->opts.max_active = 1;
    S->n_lanes = S->opts.large_dim > 0 && !S->opts.sequential ? 2 : 1;
    hipError_t e = hipGetDevice(&S->device);
    if (e == hipSuccess) e = hipMalloc(&S->arena, hbm_budget);
    if (e != hipSuccess) {
        delete S;
        return fail(ECUT_ENOMEM, std::string("server arena: ") + hipGetErrorString(e));
    }
    auto undo = [S]() {
        for (ServerLane &l : S->lanes)
            if (l.stream) hipStreamDestroy(l.stream);
        hipFree(S->arena);
        delete S;
    };
    for (int k = 0; k < S->n_lanes; ++k) {
        e = hipStreamCreateWithFlags(&S->lanes[k].stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            undo();
            return hip_fail(e, "hipStreamCreate");
        }
    }
    ecut_status rs = device_res(nullptr, nullptr, nullptr);
    if (rs != ECUT_OK) {
        undo();
        return rs;
    }
    S->alloc.init(hbm_budget);
    S->t0 = std::chrono::steady_clock::now();
    for (int k = 0; k < S->n_lanes; ++k) S->lanes[k].worker = std::thread([S, k] { S->run(k); });
    S->helper = std::thread([S] { S->help(); });
    *out = S;
    return ECUT_OK;
}

ecut_status ecut_server_submit(ecut_server *srv, const ecut_model_desc *model, const ecut_cut_desc *cut, ecut_qnum q,
                               uint64_t seed, double not_before, uint64_t *req_id) {
    if (!srv || !model || !cut) return fail(ECUT_EINVAL, "null argument");
    if (model->n_bonds < 0 || (model->n_bonds > 0 && (!model->bond_i || !model->bond_j)))
        return fail(ECUT_EINVAL, "bad bond arrays");
    if (model->n_sites <= 0 || model->n_sites > 64) return fail(ECUT_EINVAL, "bad n_sites");
    auto R = std::make_unique<Request>();
    R->own(*model);
    R->cut = *cut;
    R->q = q;
    R->seed = seed;
    R->lane = srv->n_lanes > 1 && sector_states(*model, q) >= (double)srv->opts.large_dim ? 1 : 0;
    std::lock_guard<std::mutex> g(srv->mu);
    R->id = srv->next_id++;
    R->t_submit = srv->now();
    R->not_before = not_before > 0 ? not_before : R->t_submit;
    R->t_submit = std::max(R->t_submit, R->not_before);   // latency counts from arrival
    if (req_id) *req_id = R->id;
    // keep the queue ordered by arrival time (stable for equal times)
    auto it = srv->queue.end();
    while (it != srv->queue.begin() && (*std::prev(it))->not_before > R->not_before) --it;
    srv->queue.insert(it, std::move(R));
    ++srv->n_submitted;
    srv->cv.notify_all();
    srv->cv_help.notify_one();
    return ECUT_OK;
}

ecut_status ecut_server_poll(ecut_server *srv, ecut_result *out, int32_t max, int32_t *n_done) {
    if (!srv || !n_done || (max > 0 && !out)) return fail(ECUT_EINVAL, "null argument");
    std::lock_guard<std::mutex> g(srv->mu);
    const int32_t n = (int32_t)std::min<size_t>((size_t)std::max(max, 0), srv->finished.size());
    for (int32_t k = 0; k < n; ++k) out[k] = srv->finished[k];
    srv->finished.erase(srv->finished.begin(), srv->finished.begin() + n);
    *n_done = n;
    if (srv->worker_status != ECUT_OK && n == 0)
        return fail(srv->worker_status, "server worker failed: " + srv->worker_msg);
    return n > 0 ? ECUT_OK : ECUT_EAGAIN;
}

ecut_status ecut_server_drain(ecut_server *srv) {
    if (!srv) return fail(ECUT_EINVAL, "null argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->n_finished >= srv->n_submitted || srv->worker_status != ECUT_OK; });
    if (srv->worker_status != ECUT_OK) return fail(srv->worker_status, "server worker failed: " + srv->worker_msg);
    return ECUT_OK;
}

double ecut_server_now(const ecut_server *srv) { return srv ? srv->now() : 0.0; }

void ecut_server_destroy(ecut_server *srv) {
    if (!srv) return;
    // queued requests are dropped; the helper may be building one of them,
    // so they stay alive (out of the queue) until both threads have ended
    std::deque<std::unique_ptr<Request>> dropped;
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stop = true;
        dropped.swap(srv->queue);
        srv->cv.notify_all();
        srv->cv_help.notify_all();
    }
    for (ServerLane &l : srv->lanes)
        if (l.worker.joinable()) l.worker.join();
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->cv_help.notify_all();
    }
    if (srv->helper.joinable()) srv->helper.join();
    for (ecut_sectors *s : srv->graveyard) ecut_sectors_free(s);
    srv->graveyard.clear();
    dropped.clear();
    for (ServerLane &l : srv->lanes) {
        l.stg.release();
        if (!l.stream) continue;
        hipStreamSynchronize(l.stream);
        hipStreamDestroy(l.stream);
    }
    hipFree(srv->arena);
    delete srv;
}

}  // extern "C"

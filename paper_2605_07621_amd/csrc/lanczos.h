// Batched Lanczos engine shared by ecut_lanczos_ground_state (one solve,
// optional full reorthogonalisation) and the server (many solves advancing
// together, three-term recurrence).  Internal.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "ecut_internal.h"
#include "runtime.h"

namespace ecut {

struct LzSolve {
    uint64_t uid = 0;             // unique per carved solve, never reused (keys captured graphs)
    const ecut_sectors *s = nullptr;
    int64_t n = 0;
    bool reorth = false;
    int keep = 0;                 // basis vectors per cycle (reorth)
    double *basis = nullptr;      // reorth: (keep + 1) x n
    double *ring[3] = {nullptr, nullptr, nullptr};
    double *part_apply = nullptr;
    int32_t n_apply = 0;
    double *part_norm = nullptr;
    int32_t n_chunks = 0;
    int64_t chunk = 0;            // elements per norm partial
    double *part_cgs = nullptr;   // reorth: keep x n_chunks
    double *dcoef = nullptr;      // reorth: MAX_BASIS
    double *dscale = nullptr;     // reorth: MAX_BASIS
    double *scal = nullptr;       // device scalars, see LZ_S / LZ_Z in kernels.h
    // host state
    int j = 0, total = 0, restarts = 0, max_steps = 0, max_restarts = 0;
    int pending = 0;              // launched steps not yet processed
    bool fixed = false;
    double tol = 0.0;
    std::vector<double> a, b, sc; // tridiagonal matrix; sc: scales of the basis vectors (reorth)
    double energy = 0.0, e_prev = 0.0, residual = 0.0;
    double start_norm2 = 0.0;     // |v0|^2 (read by the host when the start asks for it)
    bool done = false;
    ecut_status status = ECUT_OK;
};

// One step of a fixed set of three-term solves at fixed ring phases, captured
// as a HIP graph with its descriptors in device memory of its own; replaying
// it needs no host work but the launch.
struct LzGraph {
    hipGraphExec_t exec = nullptr;
    void *dev = nullptr;          // descriptors
    double *dev_out = nullptr;    // alpha, |w|^2 per solve
    hipStream_t st = nullptr;     // allocations are stream ordered on it
    ~LzGraph();
};

// Steps in flight: each holds the solves it advanced and pinned host room for
// their alpha, |w|^2, filled by one device-to-host copy and marked by an event.
struct LzPipe {
    struct Step {
        std::vector<LzSolve *> solves;
        double *host = nullptr;       // 2 doubles per solve: coherent pinned host memory
        double *host_dev = nullptr;   // its device address (eager steps write it directly)
        size_t cap = 0;           // solves
        hipEvent_t ev = nullptr;
        std::shared_ptr<LzGraph> graph;   // a replayed step keeps its graph alive until finished
    };
    static constexpr int DEPTH = 2;
    Step steps[DEPTH];
    int head = 0, n = 0;          // oldest in-flight step, steps in flight
    // graph replay of steps whose solves stayed the same for GRAPH_AFTER
    // launches in a row; key: (solve uid, ring phase) of every solve of the
    // step.  A solve's uid is never reused, so a graph can never be replayed
    // for another solve that took the place (and address) of a retired one.
    static constexpr int GRAPH_AFTER = 3;
    bool use_graph = false;
    std::map<std::vector<uint64_t>, std::shared_ptr<LzGraph>> graphs;
    std::vector<uint64_t> last;   // solves of the previous launch
    int same = 0;                 // launches in a row with those solves
    int graph_captures = 0, graph_replays = 0;
    ~LzPipe();
};

// doubles of device workspace for one solve
size_t lz_workspace_doubles(const ecut_sectors *s, bool reorth, int keep);
// carve the workspace (ws: lz_workspace_doubles doubles)
void lz_carve(LzSolve &L, const ecut_sectors *s, bool reorth, int keep, double *ws);
// start: x slot <- v0 (device, dim); the first scale 1/|v0| is set on the
// device.  host_norm: also synchronise st and check |v0| on the host (needed
// for the reorthogonalisation scales and to reject a zero start vector).
ecut_status lz_start(std::vector<LzSolve *> &solves, const std::vector<const double *> &v0, hipStream_t st,
                     Staging &stg, bool host_norm);
// true while a solve may take another step (not done, step budget left)
bool lz_can_launch(const LzSolve &L);
// enqueue one step for every solve that may take one (needs a free pipe slot)
ecut_status lz_launch(std::vector<LzSolve *> &solves, LzPipe &pipe, hipStream_t st, Staging &stg);
// wait for the oldest step in flight and process its scalars on the host
// (convergence, breakdown, restarts); solves already done ignore it
ecut_status lz_finish(LzPipe &pipe, hipStream_t st, Staging &stg);
// held while a step is being captured: another host thread of the process
// holds it around its own HIP calls (allocation, upload, free), which a
// stream capture in progress on the device would otherwise reject
std::mutex &lz_capture_mutex();
// one step, launched and finished (synchronises st)
ecut_status lz_step(std::vector<LzSolve *> &solves, LzPipe &pipe, hipStream_t st, Staging &stg);
// lowest eigenvalue of the final tridiagonal matrix by implicit QL
double final_energy(const LzSolve &L);
// ground-state Ritz vector of the current cycle into out (reorth only)
ecut_status lz_ritz_vector(LzSolve &L, double *out, hipStream_t st, Staging &stg);

}  // namespace ecut

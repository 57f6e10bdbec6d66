// Batched Lanczos engine shared by ecut_lanczos_ground_state (one solve,
// optional full reorthogonalisation) and the server (many solves advancing
// together, three-term recurrence).  Internal.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "ecut_internal.h"
#include "runtime.h"

namespace ecut {

struct LzSolve {
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
    double *part_cgs = nullptr;   // reorth: keep x n_chunks
    double *dcoef = nullptr;      // reorth: MAX_BASIS
    double *dscale = nullptr;     // reorth: MAX_BASIS
    double *scal = nullptr;       // device: alpha, beta^2
    // host state
    int j = 0, total = 0, restarts = 0, max_steps = 0, max_restarts = 0;
    bool fixed = false;
    double tol = 0.0;
    double s_cur = 1.0, s_prev = 0.0, beta_prev = 0.0;
    std::vector<double> a, b, sc;
    double energy = 0.0, e_prev = 0.0, residual = 0.0;
    bool done = false;
    ecut_status status = ECUT_OK;
    double host_scal[2] = {0.0, 0.0};
};

// doubles of device workspace for one solve
size_t lz_workspace_doubles(const ecut_sectors *s, bool reorth, int keep);
// carve the workspace (ws: lz_workspace_doubles doubles)
void lz_carve(LzSolve &L, const ecut_sectors *s, bool reorth, int keep, double *ws);
// start: x slot <- v0 (device, dim), computes the first scale; synchronises st
ecut_status lz_start(std::vector<LzSolve *> &solves, const std::vector<const double *> &v0, hipStream_t st,
                     Staging &stg);
// one Lanczos step for every solve that is not done; synchronises st
ecut_status lz_step(std::vector<LzSolve *> &solves, hipStream_t st, Staging &stg);
// lowest eigenvalue of the final tridiagonal matrix by implicit QL
double final_energy(const LzSolve &L);
// ground-state Ritz vector of the current cycle into out (reorth only)
ecut_status lz_ritz_vector(LzSolve &L, double *out, hipStream_t st, Staging &stg);

}  // namespace ecut

// Launch interface of the HIP kernels (kernels.hip).  Internal.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ecut_internal.h"

namespace ecut {

constexpr int ROWS_THREADS = 256;
constexpr size_t ROWS_MAX_LDS = 64 * 1024;   // generic kernel stages tiles up to this size
constexpr int HUB_THREADS = 1024;
constexpr int HUB_MAXC = 16;                 // columns per thread: d_R <= HUB_THREADS * HUB_MAXC
constexpr int HUB2_THREADS = 512;
constexpr int HUB2_M = 16;                   // element passes per thread and item
constexpr int HUB2_LOREG = 8;                // low-hop entries kept in registers
constexpr int HUB2_NB = 8;                   // left-operator neighbour loads issued together per element
constexpr int HUB3_THREADS = 512;            // threads of the fast class-tile kernel
constexpr int HUB3_M = 10;                   // element slots per thread and item in the fast kernel
constexpr int HUB3_WAVES_PER_EU = 4;         // occupancy hint of that kernel (sets its register budget)
constexpr int HUBSEG_THREADS = 512;
constexpr int HUBSEG_M = 10;                 // element slots per thread and item in the segment-tile kernel
constexpr int SLAB_W = 16;                   // columns per slab of the left-operator pass (one 128-byte line)
constexpr int SLAB_THREADS = 256;
constexpr int SPIN_THREADS = 512;
constexpr int SPIN_M = 13;                   // element slots per thread of the spin kernel
constexpr int SPIN_TILE = SPIN_THREADS * SPIN_M;
constexpr int XTAB_SLOTS = 256;               // LDS doubles of a row's folded diagonal table (2^XR_MAX)
constexpr int SPIN_MAX_FLIP = 64;            // flip-flop terms inside the right part
constexpr int SPIN_SHORT_THREADS = 256;      // two-pass one-row items of rows up to 256 x 5 amplitudes
constexpr int SPIN_SHORT_M = 5;
constexpr int SPIN_MANY_THREADS = 256;       // kernel for items of several short rows
constexpr int SPIN_MANY_TILE = 512;          // most amplitudes per such item: the default and largest tile
constexpr int HUBROW_THREADS = 1024;
constexpr int HUBROW_P = 7;                  // column pairs per thread of the whole-row Hubbard kernel
constexpr int HUBROW_P_SHORT = 4;            // the same for 512-thread groups on rows of <= 4096 columns
constexpr int HUBROW_COLS = 2 * HUBROW_P * HUBROW_THREADS;
constexpr int HUBROW_MAX_BOND = 64;
constexpr int HUBU_THREADS = 256;            // two-pass kernels: left-operator pass, one row per wave at a time
constexpr int HUBU_NB = 8;                   // neighbour-row loads issued together per lane
constexpr int HUBU_ROWS = 4;                  // rows of the row order per left-operator item
constexpr int HUBU_RMAX = 8;                  // most rows of one wave in a left-operator item
constexpr int HUBD_THREADS = 256;            // right-operator pass: one column per thread
constexpr int HUBD_NB = 8;                   // in-row gathers issued together per lane
constexpr int HUBD_MAX_SLOTS = 32;           // bonds of the down-spin hop table (held in registers)
constexpr int HUBD_BATCH_SLOTS = 16;         // the same in the batched launch (problems with more launch alone)
constexpr int HUBD_ROWS = 4;                 // default rows per right-operator item
constexpr int VEC_THREADS = 256;
constexpr int64_t VEC_CHUNK = 8192;          // elements per reduction partial
constexpr int64_t STREAM_STORE_MIN = (int64_t)32 << 20;   // elements: results of vectors this long bypass the cache
constexpr int MAX_BASIS = 1024;              // reorthogonalisation: vectors per projection call

// One vector job of the batched Lanczos kernels.
// Lanczos scalars kept on the device, per solve (scal[]): 0 alpha, 1 |w|^2,
// 2-4 reorthogonalisation norms and gate, LZ_S the scale s_j of the current
// vector (v_j = s_j w_j), LZ_Z the coefficient beta_{j-1} s_{j-1} of the
// previous one.  The apply kernels and vector jobs read them through their
// dscale pointers (scal + LZ_S).
constexpr int LZ_S = 6, LZ_Z = 7;

// Next-step job of a solve, run by k_reduce right after it wrote |w|^2 of a
// step (or of the start vector) to scal[1]: set the factors of the next step
// and copy alpha, |w|^2 to out2.
struct LzNextJob {
    double *scal;
    double *out2;            // 2 doubles for the host
    double *scales;          // nullable: scales[slot] <- new scale (reorthogonalisation basis)
    int32_t slot;
    int32_t start;           // 1: start vector (no previous vector)
};

struct VecJob {
    const double *x;
    double *y;
    int64_t n;
    double *partials;
    int32_t n_partials;
    int32_t mode;            // k_reduce: 0 -> scalars[out] = scale * sum, 1 -> sum
    double *scalars;
    int32_t out;
    int32_t coef_idx;        // k_axpy_norm: y -= scalars[coef_idx] * coef_mul * x
    double scale;
    double coef_mul;
    const double *dscale;    // nullable: scale and coef_mul are read from dscale[0]
    LzNextJob next;          // k_reduce, next.scal non-null: after the sum, the next-step job of its solve
    const double *a_partials;   // k_axpy_norm, nullable: form scalars[coef_idx] itself as
    int32_t a_n;                //   dscale[0] * sum of a_n partials (k_reduce's order and result)
    int64_t chunk;              // k_axpy_norm: elements per partial (0 = VEC_CHUNK)
};

size_t hub_lds_bytes(const ecut_sectors *s);
hipError_t set_hub_lds_limits(size_t bytes);
hipError_t launch_rows(const ProblemDev *probs_d, const ProblemDev &single, const ItemDev *items_d, int n_items,
                       int max_tile_elems, hipStream_t st);
// spin kernel with ranking tables; every problem of the launch must have
// spin_ok.  max_src: largest d_r of any block of the launch's problems.
// grid: work groups of each of the two launches (0 = min(n_items, 2048)).
hipError_t launch_spin(const ProblemDev *probs_d, const ProblemDev &single, const ItemDev *items_d, int n_items,
                       int max_tile_elems, int max_src, int grid, hipStream_t st);
hipError_t launch_hub(const ecut_sectors *s, const ProblemDev &prob, const int32_t *rows_d, int n_rows, int grid,
                      int n_xcd, hipStream_t st);
size_t hub2_lds_bytes(const ecut_sectors *s);
hipError_t launch_hub2(const ecut_sectors *s, const ProblemDev &prob, const HubItem *items_d, int n_items, int grid,
                       int n_xcd, hipStream_t st);
size_t hub3_lds_bytes(const ecut_sectors *s);
// segment tiles: grid work groups, n_xcd = 8 (items in 8 XCD chunks) or 1
hipError_t launch_hubseg(const ecut_sectors *s, const HubSegArgs &args, int grid, int n_xcd, hipStream_t st);
// two-pass kernels (variants 6 and 7): the flat left-operator pass (slab
// items; n_xcd 8 = XCD-contiguous items)
hipError_t launch_hub6_left(const HubUArgs &U, int n_xcd, hipStream_t st);
// one launch per pass over the items of n_probs Hubbard problems (device
// arrays of their arguments and of their first items, off[n_probs] = total)
hipError_t launch_hub6_batch(const HubUArgs *probs_u, const HubDArgs *probs_d, const int32_t *off_u,
                             const int32_t *off_d, int n_probs, int n_items_u, int n_items_d, hipStream_t st);
// pass 2 of the two-pass kernels alone
hipError_t launch_hubD_only(const HubDArgs &D, int n_xcd, hipStream_t st);
// split: the left operator is already in y (UP = false); slab_grid > 0 runs
// the slab pass k_upslab first, 0 leaves y as the caller wrote it
hipError_t launch_hub3(const ecut_sectors *s, const Hub3Args &args, int grid, int n_xcd, bool split, int slab_grid,
                       hipStream_t st);
int hub_blocks_per_cu(int which, size_t lds);
// whole-row Hubbard kernel: rows_d lists the rows in processing order;
// threads per work group 256, 512 or 1024 (rows of at most 2 * HUBROW_P *
// threads columns); grid 0 = as many groups as fit on n_cu compute units
hipError_t launch_hubrow(const ecut_sectors *s, const ProblemDev &prob, const int32_t *rows_d, int n_rows, int grid,
                         int n_xcd, int threads, int n_cu, hipStream_t st);
// Hubbard block whose columns are a permutation of the canonical down ranks
hipError_t launch_perm_cols(const int32_t *col_d, int64_t n_rows, int dR, const double *in, double *out, bool to_bip,
                            hipStream_t st);
hipError_t launch_perm(const ecut_sectors *s, const uint64_t *binom_d, const BlockDev *blocks_d, const double *in,
                       double *out, bool to_bip, hipStream_t st);
hipError_t launch_cdag(const CdagArgs &A, hipStream_t st);
// two-pass spin kernels: left pass over slab items, then the one-row items
// [0, n_one) and the several-row items [n_one, n_items) without the left operator
hipError_t launch_spin2(const SpinLArgs &L, const ProblemDev &P, const uint16_t *tab, const int64_t *tbase,
                        const ItemDev *items_d, int n_one, int n_items, int max_d_r, int n_xcd, bool fermion,
                        hipStream_t st);
// canonical <-> bipartite layout of the spatial Hubbard cut (with signs)
hipError_t launch_perm_hubsp(const HubSpPerm &A, const double *in, double *out, bool to_bip, hipStream_t st);
hipError_t launch_reduce(const VecJob *jobs_d, int n_jobs, hipStream_t st);
hipError_t launch_axpy_norm(const VecJob *jobs_d, const int32_t *chunk_job_d, const int32_t *chunk_idx_d, int n_chunks,
                            hipStream_t st);
// gate (nullable, device): when *gate == 0.0 the launch does nothing
hipError_t launch_multidot(const double *basis, int64_t ld, int nvec, const double *y, int64_t n, double *partials,
                           int n_chunks, hipStream_t st, const double *gate = nullptr);
hipError_t launch_multidot_reduce(const double *partials, int n_chunks, int nvec, const double *scale, double *coef,
                                  hipStream_t st, const double *gate = nullptr);
hipError_t launch_multiaxpy(const double *basis, int64_t ld, int nvec, const double *coef, const double *scale,
                            double *y, int64_t n, double *partials, int n_chunks, double sign, hipStream_t st,
                            const double *gate = nullptr);
// scal[4] = 1 if scal[3] < scal[2] / 2 else 0 (second reorthogonalisation pass needed)
hipError_t launch_dgks_gate(double *scal, hipStream_t st);
hipError_t launch_scale_copy(const double *x, double *y, int64_t n, double a, hipStream_t st);
hipError_t launch_fill_normal(double *y, int64_t n, uint64_t seed, hipStream_t st);

}  // namespace ecut

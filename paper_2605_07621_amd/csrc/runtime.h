// Internal runtime helpers shared by the ABI files.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "ecut_internal.h"
#include "kernels.h"

namespace ecut {

ecut_status hip_fail(hipError_t e, const char *what);
ecut_status device_res(int *dev, const uint64_t **binom, int *n_cu);
ecut_status launch_apply(const ecut_sectors *s, const ProblemDev &P, hipStream_t st);
int32_t apply_partial_slots(const ecut_sectors *s);        // slots the current launch writes
int32_t apply_partial_slots_max(const ecut_sectors *s);    // slots any variant may write
int32_t max_tile_elems(const ecut_sectors *s);
// key of a problem's launch tuning: device architecture and problem shape
std::string tune_shape_key(const ecut_sectors *s);

// A batched row-kernel launch over several problems: the problems (padded to
// 256 bytes), then the work items, spin-kernel items first.
struct RowsBatch {
    std::vector<char> buf;
    size_t pb = 0;
    int n_spin = 0, n_items = 0, spin_tile = 0, spin_src = 0, rows_tile = 0, first_spin = -1;
    ProblemDev spin_single{}, rows_single{};
};
void make_rows_batch(const std::vector<ProblemDev> &probs, const std::vector<ItemDev> &items,
                     const std::vector<int32_t> &tiles, RowsBatch &b);
// launch with dev = a device copy of b.buf
hipError_t launch_rows_batch(const RowsBatch &b, const void *dev, hipStream_t st);
// One row-kernel launch over the work items of several problems (two when
// spin-kernel and generic problems are mixed): copies the problem
// descriptors and the work items to a per-thread device buffer (pinned
// staging, asynchronous on `st`) and launches.  Waits for the previous use of
// the buffer before overwriting it.  tiles[k] = largest row tile of problem k.
ecut_status batch_launch_rows(const std::vector<ProblemDev> &probs, const std::vector<ItemDev> &items,
                              const std::vector<int32_t> &tiles, hipStream_t st);

// Hubbard problems of a batch that share one launch per pass of the
// two-pass kernels: their arguments (with each problem's vectors and
// epilogue) and the first item of each problem in each pass.
struct HubBatch {
    std::vector<HubUArgs> u;
    std::vector<HubDArgs> d;
    std::vector<int32_t> off_u{0}, off_d{0};
    bool empty() const { return u.empty(); }
};
// a problem joins the merged launch when its tuning selects the two-pass
// kernels (variant 6) and its down-spin table fits the batched kernel
bool hub6_batchable(const ecut_sectors *s);
// a problem that a batch launches on its own kernels (Hubbard kernels other
// than the merged two-pass launch, two-pass spin kernels)
bool own_launch(const ecut_sectors *s);
void hub6_batch_add(HubBatch &b, const ecut_sectors *s, const ProblemDev &P);
// byte offsets of the four arrays in a buffer laid out by hub6_batch_pack
struct HubBatchLayout {
    size_t u = 0, d = 0, off_u = 0, off_d = 0, bytes = 0;
};
HubBatchLayout hub6_batch_layout(const HubBatch &b, size_t base);
void hub6_batch_pack(const HubBatch &b, const HubBatchLayout &l, char *buf);
hipError_t hub6_batch_launch(const HubBatch &b, const HubBatchLayout &l, const void *dev, hipStream_t st);
// Everything one ecut_apply_H_batch launches: problems on their own
// kernels, the row-kernel queue of the spin and generic problems, the
// merged Hubbard launches, and the device image of their descriptors (the
// row queue's buffer at offset 0, then the Hubbard arrays).
struct BatchPlan {
    std::vector<ProblemDev> own;
    std::vector<const ecut_sectors *> own_s;
    RowsBatch rows;
    bool has_rows = false;
    HubBatch hub;
    HubBatchLayout hub_l;
    std::vector<char> buf;
};
ecut_status make_batch_plan(int32_t n, const ecut_sectors *const *s, const double *const *psi_d,
                            double *const *y_d, BatchPlan &pl);
// launches with dev = a device copy of pl.buf (nullable when pl.buf is empty)
ecut_status launch_batch_plan(const BatchPlan &pl, const void *dev, hipStream_t st);

// Small reusable device + pinned-host staging buffer (not thread-safe).
struct Staging {
    void *dev = nullptr;
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
    int device = -1;
    ecut_status reserve(size_t bytes);
    ecut_status wait();
    ecut_status upload(size_t bytes, hipStream_t st);   // host -> dev, then records ev
    void release();
};

}  // namespace ecut

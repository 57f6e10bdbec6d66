// Batched H*psi that allocates nothing: ecut_apply_H_batch with its launch
// descriptors in a fixed device array of this library instead of a buffer
// the library allocates.  The descriptors are written into the array by a
// small kernel that carries them as kernel arguments, so the call makes no
// allocation of any kind on the device or in pinned host memory, and every
// step of it is an ordinary kernel launch on the caller's stream.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "ecut_internal.h"
#include "kernels.h"
#include "runtime.h"

namespace ecut {
namespace {

// Descriptor bytes carried by one upload launch (kernel arguments are
// limited to 4 KiB per launch).
constexpr int PUT_BYTES = 3584;

struct PutChunk {
    unsigned char b[PUT_BYTES];
};

__global__ void k_put(unsigned char *__restrict__ dst, const PutChunk c, int n) {
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) dst[i] = c.b[i];
}

// The descriptors of one call.  Each GPU the library runs on holds its own
// copy until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[ECUT_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
std::map<int, unsigned char *> g_ptr;   // device -> address of its scratch

ecut_status scratch_ptr(unsigned char **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(ECUT_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_ptr.find(dev);
    if (it == g_ptr.end()) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ECUT_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        it = g_ptr.emplace(dev, (unsigned char *)p).first;
    }
    *out = it->second;
    return ECUT_OK;
}

}  // namespace
}  // namespace ecut

using namespace ecut;

extern "C" ecut_status ecut_apply_H_batch_noalloc(int32_t n, const ecut_sectors *const *s,
                                                  const double *const *psi_d, double *const *y_d, void *stream) {
    BatchPlan pl;
    ecut_status st = make_batch_plan(n, s, psi_d, y_d, pl);
    if (st != ECUT_OK || n == 0) return st;
    if (pl.buf.size() > ECUT_NOALLOC_SCRATCH_BYTES)
        return fail(ECUT_EINVAL, "the batch's launch descriptors take " + std::to_string(pl.buf.size()) +
                                     " bytes, more than the " + std::to_string(ECUT_NOALLOC_SCRATCH_BYTES) +
                                     " bytes of ECUT_NOALLOC_SCRATCH_BYTES");
    unsigned char *dst = nullptr;
    st = scratch_ptr(&dst);
    if (st != ECUT_OK) return st;
    const hipStream_t hs = (hipStream_t)stream;
    PutChunk c;
    for (size_t o = 0; o < pl.buf.size(); o += PUT_BYTES) {
        const int k = (int)std::min<size_t>(PUT_BYTES, pl.buf.size() - o);
        std::memcpy(c.b, pl.buf.data() + o, (size_t)k);
        hipLaunchKernelGGL(k_put, dim3(1), dim3(256), 0, hs, dst + o, c, k);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(ECUT_EDEVICE, std::string("descriptor upload: ") + hipGetErrorString(e));
    }
    return launch_batch_plan(pl, dst, hs);
}

// Entry points that allocate nothing: their kernels take their scratch
// memory from one file-scope device array instead of handle workspaces or
// allocations, for callers that cannot allocate device memory (code under
// HIP graph capture, serving loops that must not synchronise on an
// allocation, harnesses that forbid it).
//
// Every GPU the library runs on holds its own copy of the array until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol): scratch_init looks up its
// device address once per device, with that device current, and the entry
// points pass that address.  All calls on one GPU share the array, which
// keeps the last call's contents: calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <string>

#include "ddm_internal.h"

namespace ddm {

// 1 MiB: partial sums of the residual norms (2 nrhs x stencil blocks)
constexpr size_t kScratchDoubles = (size_t)1 << 17;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    g_scratch_ptr[dev] = (double *)ptr;
    return hipSuccess;
}

// device address of the scratch array on dev (null before scratch_init)
static double *scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[dev];
}

}  // namespace ddm

using namespace ddm;

int ddm_residual_noalloc(ddm_handle *h, const void *f, const void *u, void *r, int nrhs, double *norms) {
    if (!h) return DDM_EINVAL;
    if (nrhs < 1 || nrhs > h->nrhs_max || !f || !u || !norms) {
        char buf[160];
        snprintf(buf, sizeof buf, "nrhs=%d outside [1, %d], or f, u or norms null", nrhs, h->nrhs_max);
        h->err = buf;
        return DDM_EINVAL;
    }
    const size_t need = (size_t)2 * nrhs * stencil_blocks(h->plan);
    if (need > kScratchDoubles) {
        char buf[200];
        snprintf(buf, sizeof buf,
                 "ddm_residual_noalloc: %d right-hand sides on %d grid rows need %zu scratch doubles, the static "
                 "scratch holds %zu (at most %zu right-hand sides on this grid)",
                 nrhs, h->plan.G[1] * h->plan.G[2], need, kScratchDoubles,
                 kScratchDoubles / (2 * (size_t)stencil_blocks(h->plan)));
        h->err = buf;
        return DDM_EINVAL;
    }
    double *part = scratch_ptr(h->device);
    if (!part) {
        h->err = "ddm_residual_noalloc: static scratch not resolved for the handle's device";
        return DDM_ESTATE;
    }
    // every partial sum is written by the stencil kernel before the sums
    // read it: nothing in the scratch needs clearing
    hipError_t e = launch_residual_parts(h, (const double2 *)f, (const double2 *)u, (double2 *)r, nrhs, part, norms,
                                         norms + nrhs, false);
    if (e != hipSuccess) {
        char buf[160];
        snprintf(buf, sizeof buf, "HIP error %d (%s) in ddm_residual_noalloc", (int)e, hipGetErrorString(e));
        h->err = buf;
        return DDM_EHIP;
    }
    return DDM_OK;
}

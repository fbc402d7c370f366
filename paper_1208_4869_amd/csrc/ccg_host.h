// ccg_host.h -- host-side helpers shared by the solver sources: workspace
// alignment and the pinned status ring through which the host learns, a slot
// or two behind the device, that a solve has finished.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <vector>

namespace ccg {

static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Pinned, device-mapped ring of status words and the events that mark the
// end of each slot; one set per host thread and device, kept for the life of
// the process.
constexpr int kRing = 8;

struct SyncCtx {
    int device = -1;
    int* ring_h = nullptr;
    int* ring_d = nullptr;
    hipEvent_t ev[kRing];
};

static hipError_t get_sync(SyncCtx** out)
{
    thread_local std::vector<SyncCtx*> ctxs;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    for (SyncCtx* c : ctxs)
        if (c->device == dev) { *out = c; return hipSuccess; }
    SyncCtx* c = new SyncCtx;
    c->device = dev;
    e = hipHostMalloc((void**)&c->ring_h, kRing * sizeof(int),
                      hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) { delete c; return e; }
    e = hipHostGetDevicePointer((void**)&c->ring_d, c->ring_h, 0);
    if (e != hipSuccess) return e;
    for (int k = 0; k < kRing; ++k) {
        e = hipEventCreateWithFlags(&c->ev[k], hipEventDisableTiming);
        if (e != hipSuccess) return e;
    }
    ctxs.push_back(c);
    *out = c;
    return hipSuccess;
}

}  // namespace ccg

// noalloc.hip -- entry points that allocate no device memory, for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// Their scratch lives in one file-scope device array per GPU, reserved when the library is loaded
// and held until the process ends.  Host code never passes the array's name to a kernel (on the
// host that name is a stand-in, not a device address): the first call on a device looks up the
// array's address on that device with hipGetSymbolAddress and keeps it per device.  Every call on a
// GPU shares that GPU's array, so calls that overlap on one GPU (concurrent streams or threads) race
// on it; the array keeps whatever the last call left, and nothing here relies on its contents.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/dd.h"
#include "instance.hpp"
#include "kernels.hpp"

namespace {

// 16 MiB of fp32 scratch per GPU: the per-node arc probabilities of the smoothed-subproblem sweeps of
// instances up to kScratchFloats - 64 node slots (the graph-matching workload needs 2.3M).
constexpr size_t kScratchFloats = size_t(1) << 22;

static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
float *g_scratch[kMaxDevices] = {};

// The address of this GPU's scratch array (device must be current), looked up once per device.
int scratch_on(int device, float **out) {
    if (device < 0 || device >= kMaxDevices) return ddi::fail(DD_E_ARG, "device %d out of range", device);
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return ddi::fail(DD_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
        g_scratch[device] = (float *)p;
    }
    *out = g_scratch[device];
    return DD_OK;
}

}  // namespace

extern "C" {

int dd_smoothed_noalloc(dd_instance *h, float tau, int32_t flushed, float *E_out, float *p_out, void *stream) {
    if (!h || !(tau > 0.f) || !std::isfinite(tau) || (h->E && !p_out)) return ddi::fail(DD_E_ARG, "bad argument");
    const size_t need = (size_t)h->node_slots + 64;
    if (need > kScratchFloats)
        return ddi::fail(DD_E_ARG,
                         "dd_smoothed_noalloc: the instance needs %zu floats of node scratch, more than the %zu "
                         "the library holds per GPU (use dd_smoothed)",
                         need, kScratchFloats);
    int device = -1;
    HIP_TRY(hipGetDevice(&device));
    if (device != h->device)
        return ddi::fail(DD_E_ARG, "dd_smoothed_noalloc: the current device %d is not the instance's (%d)", device,
                         h->device);
    float *Qs = nullptr;
    const int st = scratch_on(device, &Qs);
    if (st) return st;
    return ddi::smoothed_sweeps(h, Qs, tau, flushed, E_out, p_out, (hipStream_t)stream);
}

}  // extern "C"

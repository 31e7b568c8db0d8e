// ct_quantize_noalloc: the quantiser with its scratch in a static device
// array instead of a caller workspace, for callers that cannot allocate
// (code under stream capture, tight serving loops, harnesses that forbid
// hipMalloc).
//
// The quantiser's only scratch is the per-plane lowpass (min, max) partials
// of its first pass. Here they live in `scratch`, a file-scope device array
// of kNoAllocPlanes planes' worth that every GPU the library runs on holds
// until the process ends. Pass 1 writes every partial that pass 2 reads, so
// nothing has to start at zero, and the contents a call leaves behind are
// never read by the next one. All calls on one GPU share its array: calls
// that overlap in time on one GPU (different streams, no ordering) race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ct_internal.h"

namespace ct {
namespace {

constexpr int kNoAllocPlanes = 1024;
constexpr size_t kScratchFloats = size_t(kNoAllocPlanes) * kMaxPart * 2;

static __device__ __align__(256) float scratch[kScratchFloats];

// Device address of `scratch` on each device, looked up once per device with
// that device current. On the host the array's name is only a stand-in for
// the symbol; kernels must be given this address.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};

int scratch_address(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CT_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return CT_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CT_ERR_HIP;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return CT_OK;
}

}  // namespace
}  // namespace ct

extern "C" int ct_quantize_noalloc(const ct_geom* geom, int32_t batch, const float* coeffs,
                                   const float* steps, int32_t steps_stride, int16_t* idx,
                                   float* side, hipStream_t stream) {
    // every argument is checked before the first HIP call
    int rc = ct::check_quantize(geom, batch, coeffs, steps, steps_stride, idx, side);
    if (rc != CT_OK || batch == 0) return rc;
    if (batch > ct::kNoAllocPlanes) return CT_ERR_WORKSPACE;
    void* p = nullptr;
    rc = ct::scratch_address(&p);
    if (rc != CT_OK) return rc;
    return ct::quantize_with_partials(geom, batch, coeffs, steps, steps_stride, idx, side, p,
                                      ct::kScratchFloats * sizeof(float), stream);
}

// Persistent work-queue kernel of the batched form (gfx950).
//
// One launch runs every stage of every stream of a plan. Each workgroup
// takes the next work item (stage, tile) from a global counter, waits until
// the stage's predecessor has finished all its tiles, runs the tile with the
// same stage code as the per-stage kernels, and counts the tile as done.
// Completion counters are released and acquired at agent scope, because the
// producer and consumer tiles may run on different XCDs, whose L2 caches are
// not coherent with each other. The grid never exceeds the number of
// workgroups that can be resident, and items are handed out in increasing
// order with every predecessor earlier, while each workgroup holds one item
// at a time: the smallest unfinished item always has its predecessor
// complete, so every wait ends.
#include "ct_batched.h"
#include "ct_quant_stages.h"

namespace ct {
namespace {

constexpr int NT = kBatchedThreads;

using LA = stage::LevelAna<4, 3, NT>;
using LS = stage::LevelSyn<4, 3, NT>;
using S1A = stage::Split<1, true, NT>;
using S2A = stage::Split<2, true, NT>;
using S1S = stage::Split<1, false, NT>;
using S2S = stage::Split<2, false, NT>;

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int SMEM = cmax(cmax(LA::SMEM, LS::SMEM), cmax(S2A::SMEM, S1A::SMEM));

__global__ __launch_bounds__(256) void reset_counters_kernel(int* counters, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        counters[i] = 0;
}

__device__ __forceinline__ int find_stage(const int* first_item, int nstages, int item) {
    int lo = 0, hi = nstages - 1;             // largest s with first_item[s] <= item
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first_item[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(NT, 4) void batched_kernel(const StageDesc* stages, const int* first_item,
                                                     int nstages, int total_items, int* done,
                                                     int* next) {
    __shared__ float smem[SMEM];
    __shared__ int item_s;
    for (;;) {
        if (threadIdx.x == 0) item_s = atomicAdd(next, 1);
        __syncthreads();
        const int item = item_s;
        __syncthreads();
        if (item >= total_items) break;
        const int s = find_stage(first_item, nstages, item);
        const int tile = item - first_item[s];
        const StageDesc& d = stages[s];
        if (d.dep >= 0) {
            if (threadIdx.x == 0) {
                // Bounded wait: by the ordering argument above the wait ends;
                // the bound only guarantees that the grid drains regardless.
                const int need = stages[d.dep].ntiles;
                for (int spins = 0; spins < (1 << 24); ++spins) {
                    if (__hip_atomic_load(done + d.dep, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= need) break;
                    __builtin_amdgcn_s_sleep(4);
                }
            }
            __syncthreads();
            __threadfence();
        }
        switch (d.type) {
            case kStLevelAna: {
                LA st(d.u.la);
                stage::run_one(st, tile, smem);
                break;
            }
            case kStLevelSyn: {
                LS st(d.u.ls);
                stage::run_one(st, tile, smem);
                break;
            }
            case kStSplit1Ana: {
                S1A st(d.u.sp, d.batch, d.lift);
                stage::run_one(st, tile, smem);
                break;
            }
            case kStSplit2Ana: {
                S2A st(d.u.sp, d.batch, d.lift);
                stage::run_one(st, tile, smem);
                break;
            }
            case kStSplit1Syn: {
                S1S st(d.u.sp, d.batch, d.lift);
                stage::run_one(st, tile, smem);
                break;
            }
            case kStSplit2Syn: {
                S2S st(d.u.sp, d.batch, d.lift);
                stage::run_one(st, tile, smem);
                break;
            }
            case kStPartial:
                qstage::lowpass_partial<NT>(d.u.q, tile, smem);
                break;
            case kStQuantize:
                qstage::quantize<NT>(d.u.q, tile, smem);
                break;
            case kStDequantize:
                qstage::dequantize<NT>(d.u.q, tile);
                break;
            default:
                break;
        }
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(done + s, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace

int batched_capacity() {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&batched_kernel),
                                                     NT, 0) != hipSuccess)
        return 0;
    return cus * per;
}

hipError_t launch_batched(const StageDesc* stages, const int* first_item, int nstages,
                          int total_items, int* counters, int grid, hipStream_t st) {
    reset_counters_kernel<<<1, 256, 0, st>>>(counters, nstages + 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    batched_kernel<<<grid, NT, 0, st>>>(stages, first_item, nstages, total_items, counters,
                                        counters + nstages);
    return hipGetLastError();
}

}  // namespace ct

// Group kernels of the batched form (gfx950).
//
// One launch runs the stages of one type at one chain position of every
// stream of a plan (forward and inverse transforms only: the split stages run
// the forward lifting, first_odd = 1, in the analysis and the inverse one,
// first_odd = 0, in the synthesis): a workgroup finds its stage among the group's stages by
// binary search over their first tiles and runs that tile with the same
// stage code as the per-stage kernels. There is no communication between
// workgroups; the launches of a plan follow each other in chain order on
// one stream.
#include "ct_batched.h"
#include "ct_quant_stages.h"
#include "ct_stream_level.h"

namespace ct {
namespace {

constexpr int NT = kBatchedThreads;

using LA = stream::StreamLevelAna<4, 3, NT>;
using LS = stream::StreamLevelSyn<4, 3, NT>;
using S1A = stream::StreamSplit<1, true, NT>;
using S2A = stream::StreamSplit<2, true, NT>;
using S1S = stream::StreamSplit<1, false, NT>;
using S2S = stream::StreamSplit<2, false, NT>;
using S3A = stream::StreamSplit<3, true, NT>;
using S3S = stream::StreamSplit<3, false, NT>;

constexpr bool quantised(int type) {
    return (type >= kStLevelAnaQ && type <= kStLevelSynQ) || type == kStSplit3AnaQ || type == kStSplit3SynQ;
}

__device__ __forceinline__ int find_stage(const int* first, int n, int tile) {
    int lo = 0, hi = n - 1;                  // largest s with first[s] <= tile
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int TYPE>
struct GroupSmem {
    static constexpr int value = (TYPE == kStLevelAna || TYPE == kStLevelAnaQ) ? LA::SMEM
                                 : (TYPE == kStLevelSyn || TYPE == kStLevelSynQ) ? LS::SMEM
                                 : (TYPE == kStPartial || TYPE == kStQuantize) ? 2 * NT / 64
                                                                               : 1;
};

template <int TYPE>
// The descriptor table is read-only for the whole launch (__restrict__), so
// the compiler may keep a stage's arguments in registers across its stores
// instead of loading them again after each one. The LP-level analysis is held
// to 128 VGPRs (four waves per SIMD, as its per-stage kernel; 64 streams
// 1.84 -> 1.81 ms).
__global__ __launch_bounds__(NT, TYPE == kStLevelAna ? 4 : 1) void group_kernel(const StageDesc* __restrict__ stages,
                                                   const int* __restrict__ first, int n) {
    __shared__ float smem[GroupSmem<TYPE>::value];
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const int s = find_stage(first, n, t);
    const int tile = t - first[s];
    const StageDesc& d = stages[s];
    constexpr bool Q = quantised(TYPE);
    if constexpr (TYPE == kStLevelAna || TYPE == kStLevelAnaQ) {
        LA st(d.u.la);
        st.template run_tile<Q>(tile, smem);
    } else if constexpr (TYPE == kStLevelSyn || TYPE == kStLevelSynQ) {
        LS st(d.u.ls);
        st.template run_tile<Q>(tile, smem);
    } else if constexpr (TYPE == kStSplit1Ana || TYPE == kStSplit1AnaQ) {
        S1A st(d.u.sp, d.batch, d.lift);
        st.template run_tile<Q, 1>(tile);
    } else if constexpr (TYPE == kStSplit2Ana || TYPE == kStSplit2AnaQ) {
        S2A st(d.u.sp, d.batch, d.lift);
        st.template run_tile<Q, 1>(tile);
    } else if constexpr (TYPE == kStSplit3Ana || TYPE == kStSplit3AnaQ) {
        S3A st(d.u.sp, d.batch, d.lift);
        st.template run_tile<Q, 1>(tile);
    } else if constexpr (TYPE == kStSplit3Syn || TYPE == kStSplit3SynQ) {
        S3S st(d.u.sp, d.batch, d.lift);
        st.template run_tile<Q, 0>(tile);
    } else if constexpr (TYPE == kStSplit1Syn || TYPE == kStSplit1SynQ) {
        S1S st(d.u.sp, d.batch, d.lift);
        st.template run_tile<Q, 0>(tile);
    } else if constexpr (TYPE == kStSplit2Syn || TYPE == kStSplit2SynQ) {
        S2S st(d.u.sp, d.batch, d.lift);
        st.template run_tile<Q, 0>(tile);
    } else if constexpr (TYPE == kStPartial) {
        qstage::lowpass_partial<NT>(d.u.q, tile, smem);
    } else if constexpr (TYPE == kStQuantize) {
        qstage::quantize<NT>(d.u.q, tile, smem);
    } else if constexpr (TYPE == kStDequantize) {
        qstage::dequantize<NT>(d.u.q, tile);
    }
}

template <int TYPE>
hipError_t launch_type(const StageDesc* stages, const int* first, int n, int tiles, hipStream_t st) {
    group_kernel<TYPE><<<tiles, NT, 0, st>>>(stages, first, n);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_group(int type, const StageDesc* stages, const int* first, int n, int tiles,
                        hipStream_t st) {
    if (n <= 0 || tiles <= 0) return hipErrorInvalidValue;
    switch (type) {
        case kStLevelAna: return launch_type<kStLevelAna>(stages, first, n, tiles, st);
        case kStLevelSyn: return launch_type<kStLevelSyn>(stages, first, n, tiles, st);
        case kStSplit1Ana: return launch_type<kStSplit1Ana>(stages, first, n, tiles, st);
        case kStSplit2Ana: return launch_type<kStSplit2Ana>(stages, first, n, tiles, st);
        case kStSplit1Syn: return launch_type<kStSplit1Syn>(stages, first, n, tiles, st);
        case kStSplit2Syn: return launch_type<kStSplit2Syn>(stages, first, n, tiles, st);
        case kStPartial: return launch_type<kStPartial>(stages, first, n, tiles, st);
        case kStQuantize: return launch_type<kStQuantize>(stages, first, n, tiles, st);
        case kStDequantize: return launch_type<kStDequantize>(stages, first, n, tiles, st);
        case kStLevelAnaQ: return launch_type<kStLevelAnaQ>(stages, first, n, tiles, st);
        case kStLevelSynQ: return launch_type<kStLevelSynQ>(stages, first, n, tiles, st);
        case kStSplit1AnaQ: return launch_type<kStSplit1AnaQ>(stages, first, n, tiles, st);
        case kStSplit2AnaQ: return launch_type<kStSplit2AnaQ>(stages, first, n, tiles, st);
        case kStSplit1SynQ: return launch_type<kStSplit1SynQ>(stages, first, n, tiles, st);
        case kStSplit2SynQ: return launch_type<kStSplit2SynQ>(stages, first, n, tiles, st);
        case kStSplit3Ana: return launch_type<kStSplit3Ana>(stages, first, n, tiles, st);
        case kStSplit3Syn: return launch_type<kStSplit3Syn>(stages, first, n, tiles, st);
        case kStSplit3AnaQ: return launch_type<kStSplit3AnaQ>(stages, first, n, tiles, st);
        case kStSplit3SynQ: return launch_type<kStSplit3SynQ>(stages, first, n, tiles, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ct

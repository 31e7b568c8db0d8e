// Per-stage kernels for gfx950: the fused LP level + DFB tree levels 1-2
// (analysis and synthesis), the deeper DFB tree levels one, two or three at a time,
// all register-streaming, and the transpose of the mirror padding.
//
// Paper section 2.1 (LP, then a DFB on each bandpass image, 9-7 filters),
// section 3.3 (half resolution per level), section 3.10 (periodic, FFT-style
// convolution). The stages themselves are in ct_stream_level.h and
// ct_stream.h: every wavefront streams one strip of rows, so a launch has
// one workgroup per four wavefront items, mapped XCD-contiguously. Built
// without FMA contraction (the stages use explicit fmaf).
#include "ct_stream_level.h"

namespace ct {
namespace {

constexpr int NT_STREAM = 256;

// One wavefront per (plane, column strip, row block). RGB: level 1 of the
// RGB encoder (the source is 8-bit RGB frames, converted on load).
template <int LO_R, int UP_R, bool Q, bool RGB = false>
__global__ __launch_bounds__(NT_STREAM) void stream_level_analysis_kernel(stage::LevelAnaArgs a) {
    using S = stream::StreamLevelAna<LO_R, UP_R, NT_STREAM>;
    __shared__ float smem[S::SMEM];
    S st(a);
    st.template run_tile<Q, RGB>(xcd_remap(blockIdx.x, gridDim.x), smem);
}

// LOWONLY: the coarsest level of the decoder, whose lowpass (only) arrives as
// indices.
template <int LO_R, int UP_R, bool Q, bool LOWONLY = false>
__global__ __launch_bounds__(NT_STREAM) void stream_level_synthesis_kernel(stage::LevelSynArgs a) {
    using S = stream::StreamLevelSyn<LO_R, UP_R, NT_STREAM>;
    __shared__ float smem[S::SMEM];
    S st(a);
    st.template run_tile<Q, LOWONLY>(xcd_remap(blockIdx.x, gridDim.x), smem);
}

// One wavefront per (plane, parent channel, column strip, row block); FO is
// the lifting's first_odd.
template <int LEVELS, bool ANA, bool Q, int FO>
__global__ __launch_bounds__(NT_STREAM) void stream_split_kernel(SplitArgs a, Lift L, int batch) {
    stream::StreamSplit<LEVELS, ANA, NT_STREAM> st(a, batch, L);
    st.template run_tile<Q, FO>(xcd_remap(blockIdx.x, gridDim.x));
}

__global__ __launch_bounds__(256) void pad_fold_kernel(CView in, int R, int C, View out, int H,
                                                       int W) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const int b = blockIdx.z;
    if (c >= W) return;
    const float* ip = in.p + b * in.plane;
    const int r2 = 2 * H - 1 - r, c2 = 2 * W - 1 - c;
    float v = ip[int64_t(r) * in.ld + c];
    if (c2 < C) v += ip[int64_t(r) * in.ld + c2];
    if (r2 < R) {
        v += ip[int64_t(r2) * in.ld + c];
        if (c2 < C) v += ip[int64_t(r2) * in.ld + c2];
    }
    out.p[b * out.plane + int64_t(r) * out.ld + c] = v;
}

}  // namespace

hipError_t launch_level_analysis(const stage::LevelAnaArgs& a, int lo_r, hipStream_t st) {
    if (a.bh <= 0 || (a.bh & 7)) return hipErrorInvalidValue;
    constexpr int waves = NT_STREAM / 64;
    const int tiles = (level_items(a.R, a.C, a.batch, a.bh) + waves - 1) / waves;
    const bool q = a.q.idx != nullptr;
    if (a.rgb) {
        // the RGB encoder: forward filters, mirror padding
        if (lo_r != 4 || a.pad_mode != kPadReflect) return hipErrorInvalidValue;
        if (q) stream_level_analysis_kernel<4, 3, true, true><<<tiles, NT_STREAM, 0, st>>>(a);
        else stream_level_analysis_kernel<4, 3, false, true><<<tiles, NT_STREAM, 0, st>>>(a);
        return hipGetLastError();
    }
    if (lo_r == 4 && !q) stream_level_analysis_kernel<4, 3, false><<<tiles, NT_STREAM, 0, st>>>(a);
    else if (lo_r == 4) stream_level_analysis_kernel<4, 3, true><<<tiles, NT_STREAM, 0, st>>>(a);
    else if (lo_r == 3 && !q) stream_level_analysis_kernel<3, 4, false><<<tiles, NT_STREAM, 0, st>>>(a);
    else return hipErrorInvalidValue;   // the transposes never quantise
    return hipGetLastError();
}

hipError_t launch_level_synthesis(const stage::LevelSynArgs& a, int lo_r, hipStream_t st) {
    if (a.bh <= 0 || (a.bh & 7)) return hipErrorInvalidValue;
    constexpr int waves = NT_STREAM / 64;
    const int tiles = (level_items(a.R, a.C, a.batch, a.bh) + waves - 1) / waves;
    const bool q = a.q.idx != nullptr || a.lq.idx != nullptr;
    if (lo_r == 4 && !q) stream_level_synthesis_kernel<4, 3, false><<<tiles, NT_STREAM, 0, st>>>(a);
    else if (lo_r == 4 && !a.q.idx) stream_level_synthesis_kernel<4, 3, true, true><<<tiles, NT_STREAM, 0, st>>>(a);
    else if (lo_r == 4) stream_level_synthesis_kernel<4, 3, true><<<tiles, NT_STREAM, 0, st>>>(a);
    else if (lo_r == 3 && !q) stream_level_synthesis_kernel<3, 4, false><<<tiles, NT_STREAM, 0, st>>>(a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int LEVELS, bool ANA>
static hipError_t launch_split(const SplitArgs& a, Lift lift, int batch, hipStream_t st) {
    if (a.bh <= 0 || a.bh % stream_row_align(LEVELS)) return hipErrorInvalidValue;
    if ((a.Rj & 3) || (a.Cj & 3)) return hipErrorInvalidValue;   // channel rows of even width
    constexpr int waves = NT_STREAM / 64;
    const int tiles = (stream_items(a, batch, LEVELS) + waves - 1) / waves;
    if (a.q.idx && lift.first_odd) stream_split_kernel<LEVELS, ANA, true, 1><<<tiles, NT_STREAM, 0, st>>>(a, lift, batch);
    else if (a.q.idx) stream_split_kernel<LEVELS, ANA, true, 0><<<tiles, NT_STREAM, 0, st>>>(a, lift, batch);
    else if (lift.first_odd) stream_split_kernel<LEVELS, ANA, false, 1><<<tiles, NT_STREAM, 0, st>>>(a, lift, batch);
    else stream_split_kernel<LEVELS, ANA, false, 0><<<tiles, NT_STREAM, 0, st>>>(a, lift, batch);
    return hipGetLastError();
}

hipError_t launch_dfb_split_analysis(const SplitArgs& a, Lift lift, int batch, hipStream_t st) {
    return launch_split<1, true>(a, lift, batch, st);
}
hipError_t launch_dfb_split_synthesis(const SplitArgs& a, Lift lift, int batch, hipStream_t st) {
    return launch_split<1, false>(a, lift, batch, st);
}
hipError_t launch_dfb_split2_analysis(const SplitArgs& a, Lift lift, int batch, hipStream_t st) {
    return launch_split<2, true>(a, lift, batch, st);
}
hipError_t launch_dfb_split2_synthesis(const SplitArgs& a, Lift lift, int batch, hipStream_t st) {
    return launch_split<2, false>(a, lift, batch, st);
}
hipError_t launch_dfb_split3_analysis(const SplitArgs& a, Lift lift, int batch, hipStream_t st) {
    return launch_split<3, true>(a, lift, batch, st);
}
hipError_t launch_dfb_split3_synthesis(const SplitArgs& a, Lift lift, int batch, hipStream_t st) {
    return launch_split<3, false>(a, lift, batch, st);
}

hipError_t launch_pad_fold(CView in, int R, int C, View out, int H, int W, int batch,
                           hipStream_t st) {
    dim3 grid((W + 255) / 256, H, batch);
    pad_fold_kernel<<<grid, 256, 0, st>>>(in, R, C, out, H, W);
    return hipGetLastError();
}

}  // namespace ct

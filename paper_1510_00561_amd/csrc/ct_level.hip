// Per-stage persistent kernels for gfx950: the fused LP level + DFB tree
// levels 1-2 (analysis and synthesis), the deeper DFB tree levels one or two
// at a time, and the transpose of the mirror padding.
//
// Paper section 2.1 (LP, then a DFB on each bandpass image, 9-7 filters),
// section 3.3 (half resolution per level), section 3.10 (periodic, FFT-style
// convolution). The tile stages themselves are in ct_stages.h. Each kernel
// launches at most as many workgroups as can be resident; every workgroup
// walks an XCD-contiguous range of tiles and prefetches the next tile's
// loads into registers while the current one computes.
#include <mutex>

#include "ct_stages.h"

namespace ct {
namespace {

constexpr int NT_LEVEL = 512;
constexpr int NT_SPLIT = 512;

template <int LO_R, int UP_R>
__global__ __launch_bounds__(NT_LEVEL, 4) void level_analysis_kernel(stage::LevelAnaArgs a) {
    using S = stage::LevelAna<LO_R, UP_R, NT_LEVEL>;
    __shared__ float smem[S::SMEM];
    S st(a);
    stage::tile_loop(st, smem);
}

template <int LO_R, int UP_R>
__global__ __launch_bounds__(NT_LEVEL, 4) void level_synthesis_kernel(stage::LevelSynArgs a) {
    using S = stage::LevelSyn<LO_R, UP_R, NT_LEVEL>;
    __shared__ float smem[S::SMEM];
    S st(a);
    stage::tile_loop(st, smem);
}

template <int LEVELS, bool ANA>
__global__ __launch_bounds__(NT_SPLIT) void split_kernel(SplitArgs a, Lift L, int batch) {
    using S = stage::Split<LEVELS, ANA, NT_SPLIT>;
    __shared__ float smem[S::SMEM];
    S st(a, batch, L);
    stage::tile_loop(st, smem);
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

// Resident workgroups of `kernel` on the current device (cached per kernel
// and device; host queries only, no allocation).
int resident_blocks(const void* kernel, int threads) {
    struct Key {
        const void* k;
        int dev;
    };
    static std::mutex mu;
    static Key keys[64];
    static int vals[64];
    static int n = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lock(mu);
    for (int i = 0; i < n; ++i)
        if (keys[i].k == kernel && keys[i].dev == dev) return vals[i];
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess) return 0;
    const int total = cus * (per > 0 ? per : 1);
    if (n < 64) {
        keys[n] = Key{kernel, dev};
        vals[n] = total;
        ++n;
    }
    return total;
}

int grid_for(const void* kernel, int threads, int tiles) {
    const int cap = resident_blocks(kernel, threads);
    if (cap <= 0) return tiles;
    return tiles < cap ? tiles : cap;
}

int split_tile_count(const SplitArgs& a, int batch, int tr, int tc) {
    const int t = a.t;
    const int th = (((a.Rj >> (t - 2)) + tr - 1) / tr) * (((a.Cj >> 1) + tc - 1) / tc);
    const int tv = (((a.Cj >> (t - 2)) + tr - 1) / tr) * (((a.Rj >> 1) + tc - 1) / tc);
    return (1 << (t - 2)) * (th + tv) * batch;
}

}  // namespace

hipError_t launch_lp_dfb12_analysis(CView src, int src_h, int src_w, int pad_mode, int R, int C,
                                    View c_out, Quad out, Taps5 lo, int lo_r, Taps5 up, int up_r,
                                    Lift lift, int batch, hipStream_t st) {
    stage::LevelAnaArgs a{src, src_h, src_w, pad_mode, R, C, c_out, out, lo, up, lift, batch};
    const int tiles = ((C + 63) / 64) * ((R + 63) / 64) * batch;
    if (lo_r == 4 && up_r == 3) {
        const void* k = reinterpret_cast<const void*>(&level_analysis_kernel<4, 3>);
        level_analysis_kernel<4, 3><<<grid_for(k, NT_LEVEL, tiles), NT_LEVEL, 0, st>>>(a);
    } else if (lo_r == 3 && up_r == 4) {
        const void* k = reinterpret_cast<const void*>(&level_analysis_kernel<3, 4>);
        level_analysis_kernel<3, 4><<<grid_for(k, NT_LEVEL, tiles), NT_LEVEL, 0, st>>>(a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dfb12_lp_synthesis(Quad in, CView c_in, int R, int C, View x_out, int out_h,
                                     int out_w, Taps5 lo, int lo_r, Taps5 up, int up_r, Lift lift,
                                     int batch, hipStream_t st) {
    stage::LevelSynArgs a{in, c_in, R, C, x_out, out_h, out_w, lo, up, lift, batch};
    const int tiles = ((C + 63) / 64) * ((R + 63) / 64) * batch;
    if (lo_r == 4 && up_r == 3) {
        const void* k = reinterpret_cast<const void*>(&level_synthesis_kernel<4, 3>);
        level_synthesis_kernel<4, 3><<<grid_for(k, NT_LEVEL, tiles), NT_LEVEL, 0, st>>>(a);
    } else if (lo_r == 3 && up_r == 4) {
        const void* k = reinterpret_cast<const void*>(&level_synthesis_kernel<3, 4>);
        level_synthesis_kernel<3, 4><<<grid_for(k, NT_LEVEL, tiles), NT_LEVEL, 0, st>>>(a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int LEVELS, bool ANA>
static hipError_t launch_split(const SplitArgs& a, Lift lift, int batch, hipStream_t st) {
    const int tiles = split_tile_count(a, batch, LEVELS == 1 ? 32 : 64, 64);
    const void* k = reinterpret_cast<const void*>(&split_kernel<LEVELS, ANA>);
    split_kernel<LEVELS, ANA><<<grid_for(k, NT_SPLIT, tiles), NT_SPLIT, 0, st>>>(a, lift, batch);
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

hipError_t launch_pad_fold(CView in, int R, int C, View out, int H, int W, int batch,
                           hipStream_t st) {
    dim3 grid((W + 255) / 256, H, batch);
    pad_fold_kernel<<<grid, 256, 0, st>>>(in, R, C, out, H, W);
    return hipGetLastError();
}

}  // namespace ct

// Colour, chroma and K-frame lowpass kernels for gfx950: one thread per four
// pixels (or per lowpass column), blocks mapped XCD-contiguously so that the
// image rows sharing chroma samples stay in one L2. Built without FMA
// contraction. The per-thread bodies are in ct_color_stages.h.
//
// A thread's group of four pixels is 12 bytes of 8-bit RGB, or 48 bytes of
// float RGB. A wavefront whose 64 groups are all full moves that interleaved
// data as contiguous runs instead (lane l takes element l + 64 s of the
// wave's span), exchanged through a wave-private LDS block, so every global
// access of the wave covers one contiguous 256-byte (words) or 1 KB
// (float4) range.
#include "ct_color.h"
#include "ct_color_stages.h"
#include "ct_kernels.h"

namespace ct {
namespace {

constexpr int NT = 256;
constexpr int NT_DIFF = 64;   // small lowpass: spread its columns over more CUs

constexpr int kSpan = 3 * 64;   // words (forward) or float4 (inverse) per full wave
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(NT) void rgb_to_ycocg_kernel(const uint8_t* __restrict__ rgb,
                                                          float* __restrict__ y,
                                                          float* __restrict__ co,
                                                          float* __restrict__ cg,
                                                          color::Frame f) {
    __shared__ uint32_t stage[NT / 64][kSpan];
    const uint32_t t = uint32_t(xcd_remap(blockIdx.x, gridDim.x)) * NT + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63, t0 = t - lane;
    if ((t0 + 64) * color::kPix <= f.P) {   // wave-uniform: all 64 groups full
        const uint32_t* src = reinterpret_cast<const uint32_t*>(rgb) + 3 * t0;
        const uint32_t v0 = src[lane], v1 = src[lane + 64], v2 = src[lane + 128];
        uint32_t* st = stage[threadIdx.x >> 6];
        st[lane] = v0;
        st[lane + 64] = v1;
        st[lane + 128] = v2;
        wave_sync();
        const uint32_t w[3] = {st[3 * lane], st[3 * lane + 1], st[3 * lane + 2]};
        color::rgb_to_ycocg_words(t, w, y, co, cg, f);
    } else {
        color::rgb_to_ycocg(t, rgb, y, co, cg, f);
    }
}

template <int K>
__global__ __launch_bounds__(NT) void ycocg_to_rgb_kernel(const float* __restrict__ y,
                                                          const float* __restrict__ co,
                                                          const float* __restrict__ cg,
                                                          float* __restrict__ rgb, color::Frame f,
                                                          float rn) {
    __shared__ float4 stage[NT / 64][kSpan];
    const uint32_t t = uint32_t(xcd_remap(blockIdx.x, gridDim.x)) * NT + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63, t0 = t - lane;
    float out[3 * color::kPix];
    const uint32_t cnt = color::rgb_group<K>(t, y, co, cg, f, rn, out);
    if ((t0 + 64) * color::kPix <= f.P) {   // wave-uniform: all 64 groups full
        float4* st = stage[threadIdx.x >> 6];
        st[3 * lane] = make_float4(out[0], out[1], out[2], out[3]);
        st[3 * lane + 1] = make_float4(out[4], out[5], out[6], out[7]);
        st[3 * lane + 2] = make_float4(out[8], out[9], out[10], out[11]);
        wave_sync();
        // the output is written once and not read back here: streaming stores
        const v4f* sv = reinterpret_cast<const v4f*>(st);
        v4f* dst = reinterpret_cast<v4f*>(rgb) + 3 * size_t(t0);
        __builtin_nontemporal_store(sv[lane], dst + lane);
        __builtin_nontemporal_store(sv[lane + 64], dst + lane + 64);
        __builtin_nontemporal_store(sv[lane + 128], dst + lane + 128);
    } else if (cnt) {
        color::store_rgb(t, cnt, out, rgb);
    }
}

__global__ __launch_bounds__(NT_DIFF) void lowpass_diff_kernel(int16_t* idx, uint32_t plane,
                                                               int rows, int cols, int batch,
                                                               int inverse) {
    color::lowpass_diff(blockIdx.x * NT_DIFF + threadIdx.x, idx, plane, rows, cols, batch,
                        inverse != 0);
}

unsigned groups(uint32_t P) { return (P + color::kPix - 1) / color::kPix; }

}  // namespace

hipError_t launch_rgb_to_ycocg(const uint8_t* rgb, float* y, float* co, float* cg,
                               const color::Frame& f, hipStream_t st) {
    const unsigned blocks = (groups(f.P) + NT - 1) / NT;
    rgb_to_ycocg_kernel<<<blocks, NT, 0, st>>>(rgb, y, co, cg, f);
    return hipGetLastError();
}

hipError_t launch_ycocg_to_rgb(const float* y, const float* co, const float* cg, float* rgb,
                               const color::Frame& f, hipStream_t st) {
    const unsigned blocks = (groups(f.P) + NT - 1) / NT;
    const float rn = 1.0f / float(f.n);
    switch (color::window_cols(f.n)) {
        case 5: ycocg_to_rgb_kernel<5><<<blocks, NT, 0, st>>>(y, co, cg, rgb, f, rn); break;
        case 4: ycocg_to_rgb_kernel<4><<<blocks, NT, 0, st>>>(y, co, cg, rgb, f, rn); break;
        default: ycocg_to_rgb_kernel<3><<<blocks, NT, 0, st>>>(y, co, cg, rgb, f, rn); break;
    }
    return hipGetLastError();
}

hipError_t launch_lowpass_diff(int16_t* idx, uint32_t plane, int rows, int cols, int batch,
                               bool inverse, hipStream_t st) {
    const unsigned blocks = (unsigned(batch) * unsigned(cols) + NT_DIFF - 1) / NT_DIFF;
    lowpass_diff_kernel<<<blocks, NT_DIFF, 0, st>>>(idx, plane, rows, cols, batch, inverse ? 1 : 0);
    return hipGetLastError();
}

}  // namespace ct

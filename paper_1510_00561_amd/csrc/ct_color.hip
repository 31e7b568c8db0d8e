// Colour, chroma and K-frame lowpass kernels for gfx950: one thread per four
// pixels (or per lowpass column), blocks mapped XCD-contiguously so that the
// image rows sharing chroma samples stay in one L2. Built without FMA
// contraction. The per-thread bodies are in ct_color_stages.h.
#include "ct_color.h"
#include "ct_color_stages.h"
#include "ct_kernels.h"

namespace ct {
namespace {

constexpr int NT = 256;
constexpr int NT_DIFF = 64;   // small lowpass: spread its columns over more CUs

__global__ __launch_bounds__(NT) void rgb_to_ycocg_kernel(const uint8_t* __restrict__ rgb,
                                                          float* __restrict__ y,
                                                          float* __restrict__ co,
                                                          float* __restrict__ cg,
                                                          color::Frame f) {
    const uint32_t t = uint32_t(xcd_remap(blockIdx.x, gridDim.x)) * NT + threadIdx.x;
    color::rgb_to_ycocg(t, rgb, y, co, cg, f);
}

template <int K>
__global__ __launch_bounds__(NT) void ycocg_to_rgb_kernel(const float* __restrict__ y,
                                                          const float* __restrict__ co,
                                                          const float* __restrict__ cg,
                                                          float* __restrict__ rgb, color::Frame f,
                                                          float rn) {
    const uint32_t t = uint32_t(xcd_remap(blockIdx.x, gridDim.x)) * NT + threadIdx.x;
    color::ycocg_to_rgb<K>(t, y, co, cg, rgb, f, rn);
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

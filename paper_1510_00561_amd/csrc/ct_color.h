// Launchers of the colour, chroma and K-frame lowpass kernels (ct_color.hip).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace ct {
namespace color {
struct Frame;
}

hipError_t launch_rgb_to_ycocg(const uint8_t* rgb, float* y, float* co, float* cg,
                               const color::Frame& f, hipStream_t st);
hipError_t launch_ycocg_to_rgb(const float* y, const float* co, const float* cg, float* rgb,
                               const color::Frame& f, hipStream_t st);
hipError_t launch_lowpass_diff(int16_t* idx, uint32_t plane, int rows, int cols, int batch,
                               bool inverse, hipStream_t st);

}  // namespace ct

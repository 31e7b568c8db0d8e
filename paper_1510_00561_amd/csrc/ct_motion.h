// Launcher of the block-matching motion search (ct_motion.hip).
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

namespace ct {

constexpr int kMotionBlock = 16;   // block side (paper section 3.2)
constexpr int kMotionMaxW = 16;    // largest search range served

struct MotionArgs {
    const float* cur;     // [B][H][W] current luminance planes
    const float* prev;    // [B][H][W] previous luminance planes
    int16_t* mv;          // [B][nby][nbx][2] (dy, dx)
    int32_t* ssd;         // [B][nby][nbx] or null
    int H, W, w, nby, nbx, items;
    int lds_per_wave;     // 32-bit words of LDS per wavefront
};

size_t motion_lds_per_wave(int w);
hipError_t launch_motion_search(const MotionArgs& a, hipStream_t st);

}  // namespace ct

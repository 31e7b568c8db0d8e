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
    // LDS layout per wavefront, in 32-bit words: the even-column pairs of
    // the window at 0 with row pitch `rp`, the odd-column pairs at `odd_off`
    // (same pitch), the block's pairs at `cur_off`, `lds_per_wave` in all
    int rp, odd_off, cur_off, lds_per_wave;
};

// Fills the LDS layout of `a` for its search range a.w.
void motion_layout(MotionArgs* a);
hipError_t launch_motion_search(const MotionArgs& a, hipStream_t st);

}  // namespace ct

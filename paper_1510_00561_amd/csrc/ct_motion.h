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

// Work of one block: tasks of two candidates each, (dy, sc) and (dy, sc + 2)
// with sc = dx + w and sc mod 4 in {0, 1}; motion_tasks_per_row(w) tasks per
// window row cover every sc in [0, 2w] once. Task t is window row `row`
// (dy = row - w) and first column offset `sa`.
__host__ __device__ inline int motion_tasks_per_row(int w) {
    const int side = 2 * w + 1, rem = side % 4;
    return 2 * (side / 4) + (rem < 2 ? rem : 2);
}
__host__ __device__ inline int motion_tasks(int w) { return (2 * w + 1) * motion_tasks_per_row(w); }
__host__ __device__ inline void motion_task(int w, int t, int* row, int* sa) {
    const int tpr = motion_tasks_per_row(w);
    *row = t / tpr;
    const int u = t - *row * tpr;
    *sa = 4 * (u >> 1) + (u & 1);
}
// Passes over the tasks of a full block: a last pass of at most 32 tasks runs
// as half-tasks on lane pairs (lanes 2i and 2i + 1 take rows 0-7 and 8-15 of
// task 64 nfull + i), flagged by `split`.
__host__ __device__ inline void motion_passes(int w, bool full, int* nfull, int* tail, bool* split) {
    const int nt = motion_tasks(w);
    *nfull = nt / 64;
    *tail = nt - 64 * *nfull;
    *split = full && *tail > 0 && *tail <= 32;
}
hipError_t launch_motion_search(const MotionArgs& a, hipStream_t st);

}  // namespace ct

// C ABI of the block-matching motion search: validation on the host, then
// one launch (kernel in ct_motion.hip).
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>

#include "ct_motion.h"
#include "ct_plan_internal.h"

namespace {

bool fault_injected() {
    const char* f = getenv("CT_FAULT_INJECT");
    return f && strcmp(f, "launch") == 0;
}

}  // namespace

extern "C" {

int ct_motion_search(int32_t batch, int32_t height, int32_t width, int32_t w, const float* cur,
                     const float* prev, int16_t* mv, int32_t* ssd, hipStream_t stream) {
    if (batch < 0 || height < 1 || width < 1 || w < 1 || w > ct::kMotionMaxW) return CT_ERR_ARG;
    const int64_t pixels = int64_t(batch) * height * width;
    if (pixels >= (int64_t(1) << 31)) return CT_ERR_ARG;
    if (batch == 0) return CT_OK;
    if (!cur || !prev || !mv) return CT_ERR_ARG;
    if (fault_injected()) return CT_ERR_HIP;
    ct::MotionArgs a;
    a.cur = cur;
    a.prev = prev;
    a.mv = mv;
    a.ssd = ssd;
    a.H = height;
    a.W = width;
    a.w = w;
    a.nby = (height + ct::kMotionBlock - 1) / ct::kMotionBlock;
    a.nbx = (width + ct::kMotionBlock - 1) / ct::kMotionBlock;
    a.items = int(int64_t(batch) * a.nby * a.nbx);
    ct::motion_layout(&a);
    // compulsory bytes: both planes read once, the vectors (and sums) written once
    const double bytes = 8.0 * double(pixels) + a.items * (4.0 + (ssd ? 4.0 : 0.0));
    CT_PROFILED("motion_search", bytes, ct::launch_motion_search(a, stream), stream);
    return CT_OK;
}

int ct_motion_layout_query(int32_t w, int32_t* layout, int32_t* rows, int32_t* sa, int32_t cap) {
    if (w < 1 || w > ct::kMotionMaxW || !layout || cap < 0 || (cap > 0 && (!rows || !sa))) return CT_ERR_ARG;
    ct::MotionArgs a;
    memset(&a, 0, sizeof(a));
    a.w = w;
    ct::motion_layout(&a);
    int nfull, tail;
    bool split;
    ct::motion_passes(w, true, &nfull, &tail, &split);
    layout[0] = a.rp;
    layout[1] = a.odd_off;
    layout[2] = a.cur_off;
    layout[3] = a.lds_per_wave;
    layout[4] = ct::motion_tasks_per_row(w);
    layout[5] = split ? 1 : 0;
    const int nt = ct::motion_tasks(w);
    for (int t = 0; t < nt && t < cap; ++t) ct::motion_task(w, t, rows + t, sa + t);
    return nt;
}

}  // extern "C"

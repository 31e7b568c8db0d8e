// C ABI of the colour, chroma and K-frame lowpass stages: argument
// validation on the host, then one launch each (kernels in ct_color.hip).
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>

#include "ct_color.h"
#include "ct_color_stages.h"
#include "ct_plan_internal.h"

namespace {

constexpr int64_t kMaxElems = int64_t(1) << 31;

// CT_FAULT_INJECT=launch makes every call fail as a failed launch would,
// after validation and before any launch (as in the transform calls).
bool fault_injected() {
    const char* f = getenv("CT_FAULT_INJECT");
    return f && strcmp(f, "launch") == 0;
}

bool aligned(const void* p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

// Validates the frame sizes and fills `f`; 3 * P (the RGB elements) must stay
// below 2^31 so that every offset fits in 32 bits.
int frame(int32_t batch, int32_t height, int32_t width, int32_t n, ct::color::Frame* f) {
    if (batch < 0 || height < 1 || width < 1 || n < 1 || n > CT_MAX_CHROMA_FACTOR) return CT_ERR_ARG;
    const int64_t P = int64_t(batch) * height * width;
    if (3 * P >= kMaxElems) return CT_ERR_ARG;
    f->H = height;
    f->W = width;
    f->n = n;
    f->Hc = (height + n - 1) / n;
    f->Wc = (width + n - 1) / n;
    f->P = uint32_t(P);
    return CT_OK;
}

}  // namespace

extern "C" {

int ct_rgb_to_ycocg(int32_t batch, int32_t height, int32_t width, int32_t n, const uint8_t* rgb,
                    float* y, float* co, float* cg, hipStream_t stream) {
    ct::color::Frame f;
    const int rc = frame(batch, height, width, n, &f);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!rgb || !y || !co || !cg) return CT_ERR_ARG;
    if (!aligned(rgb, 4) || !aligned(y, 16)) return CT_ERR_ARG;
    if (fault_injected()) return CT_ERR_HIP;
    const double chroma = 2.0 * batch * f.Hc * f.Wc * sizeof(float);
    const double bytes = double(f.P) * (3 + sizeof(float)) + chroma;
    CT_PROFILED("rgb_to_ycocg", bytes, ct::launch_rgb_to_ycocg(rgb, y, co, cg, f, stream), stream);
    return CT_OK;
}

int ct_ycocg_to_rgb(int32_t batch, int32_t height, int32_t width, int32_t n, const float* y,
                    const float* co, const float* cg, float* rgb, hipStream_t stream) {
    ct::color::Frame f;
    const int rc = frame(batch, height, width, n, &f);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!rgb || !y || !co || !cg) return CT_ERR_ARG;
    if (!aligned(rgb, 16) || !aligned(y, 16)) return CT_ERR_ARG;
    if (fault_injected()) return CT_ERR_HIP;
    const double chroma = 2.0 * batch * f.Hc * f.Wc * sizeof(float);
    const double bytes = double(f.P) * 4 * sizeof(float) + chroma;
    CT_PROFILED("ycocg_to_rgb", bytes, ct::launch_ycocg_to_rgb(y, co, cg, rgb, f, stream), stream);
    return CT_OK;
}

int ct_lowpass_diff(const ct_geom* geom, int32_t batch, int16_t* idx, int32_t inverse,
                    hipStream_t stream) {
    if (!geom || batch < 0 || batch > 65535) return CT_ERR_ARG;
    ct::Geometry g;
    const int rc = ct::resolve(geom, &g);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!idx) return CT_ERR_ARG;
    if (int64_t(batch) * g.ncoef >= kMaxElems) return CT_ERR_ARG;
    if (fault_injected()) return CT_ERR_HIP;
    const int rows = g.R >> g.J, cols = g.C >> g.J;
    const double bytes = 2.0 * batch * double(rows) * cols * sizeof(int16_t);
    CT_PROFILED(inverse ? "lowpass_undiff" : "lowpass_diff", bytes,
                ct::launch_lowpass_diff(idx, uint32_t(g.ncoef), rows, cols, batch, inverse != 0,
                                        stream),
                stream);
    return CT_OK;
}

}  // extern "C"

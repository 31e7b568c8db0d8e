// Runs the per-thread bodies of the colour, chroma and K-frame stages
// (ct_color_stages.h) on the CPU over exactly sized buffers, for every
// thread of each launch, so that an address sanitizer catches any access
// outside the buffers and an undefined-behaviour sanitizer any overflow.
// It also checks that every output element is written: Y, the kept chroma
// samples and the RGB output start as NaN and must all end finite.
// Exit status 0 on success.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ct_color_stages.h"

using ct::color::Frame;

static Frame frame(int B, int H, int W, int n) {
    Frame f;
    f.H = H;
    f.W = W;
    f.n = n;
    f.Hc = (H + n - 1) / n;
    f.Wc = (W + n - 1) / n;
    f.P = uint32_t(B) * H * W;
    return f;
}

template <int K>
static void back(const Frame& f, const float* y, const float* co, const float* cg, float* rgb,
                 uint32_t groups) {
    const float rn = 1.0f / float(f.n);
    for (uint32_t t = 0; t < groups + 3; ++t)   // a few threads past the end, as a grid would have
        ct::color::ycocg_to_rgb<K>(t, y, co, cg, rgb, f, rn);
}

static int run(int B, int H, int W, int n) {
    const Frame f = frame(B, H, W, n);
    const uint32_t groups = (f.P + ct::color::kPix - 1) / ct::color::kPix;
    // exact sizes (rgb rounded up to whole 4-byte words, as the API requires
    // 4-byte alignment of the start only: the full-group path reads 12 bytes
    // of a group that lies wholly inside the batch)
    std::vector<uint8_t> rgb(3 * size_t(f.P));
    for (size_t i = 0; i < rgb.size(); ++i) rgb[i] = uint8_t((i * 37 + 11) & 255);
    std::vector<float> y(f.P, NAN), co(size_t(B) * f.Hc * f.Wc, NAN), cg(co.size(), NAN);
    for (uint32_t t = 0; t < groups + 3; ++t)
        ct::color::rgb_to_ycocg(t, rgb.data(), y.data(), co.data(), cg.data(), f);
    for (float v : y)
        if (!std::isfinite(v)) return 1;
    for (size_t i = 0; i < co.size(); ++i)
        if (!std::isfinite(co[i]) || !std::isfinite(cg[i])) return 2;
    std::vector<float> out(3 * size_t(f.P), NAN);
    switch (ct::color::window_cols(n)) {
        case 5: back<5>(f, y.data(), co.data(), cg.data(), out.data(), groups); break;
        case 4: back<4>(f, y.data(), co.data(), cg.data(), out.data(), groups); break;
        default: back<3>(f, y.data(), co.data(), cg.data(), out.data(), groups); break;
    }
    for (float v : out)
        if (!std::isfinite(v)) return 3;
    if (n == 1)   // exact round trip of 8-bit RGB at full chroma
        for (size_t i = 0; i < out.size(); ++i)
            if (out[i] != float(rgb[i])) return 4;
    // K-frame filter on a lowpass of rows x cols per plane, planes `plane` apart
    const int rows = (H + 7) / 8, cols = (W + 7) / 8;
    const uint32_t plane = uint32_t(rows * cols + 5);
    std::vector<int16_t> idx(size_t(B) * plane);
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = int16_t((i * 7919) & 0xFFFF);
    const std::vector<int16_t> orig = idx;
    const uint32_t threads = uint32_t(B) * cols + 64;
    for (uint32_t t = 0; t < threads; ++t) ct::color::lowpass_diff(t, idx.data(), plane, rows, cols, B, false);
    for (uint32_t t = 0; t < threads; ++t) ct::color::lowpass_diff(t, idx.data(), plane, rows, cols, B, true);
    if (idx != orig) return 5;
    return 0;
}

int main() {
    const int shapes[][4] = {
        {1, 1, 1, 1},   {2, 1, 7, 1},   {1, 5, 1, 2},    {3, 4, 4, 2},    {2, 24, 36, 2},
        {1, 30, 41, 3}, {2, 17, 23, 4}, {1, 64, 64, 8},  {3, 70, 90, 4},  {1, 13, 200, 64},
        {2, 9, 9, 5},   {1, 480, 640, 4}, {4, 33, 65, 1}, {1, 100, 3, 7},
    };
    for (const auto& s : shapes) {
        const int rc = run(s[0], s[1], s[2], s[3]);
        if (rc != 0) {
            std::printf("failed: B=%d H=%d W=%d n=%d (check %d)\n", s[0], s[1], s[2], s[3], rc);
            return rc;
        }
    }
    std::printf("colour stage indexing: %zu shapes clean\n", sizeof(shapes) / sizeof(shapes[0]));
    return 0;
}

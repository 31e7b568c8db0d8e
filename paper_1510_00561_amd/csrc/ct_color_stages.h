// Per-thread bodies of the colour, chroma and K-frame lowpass stages.
//
// Paper section 2.3 (Table I: RGB to YCoCg, equations (1)-(3), and back,
// equations (4)-(6)); section 3.1 (chroma kept at every N-th sample in both
// directions and offset by +127; the decoder removes the offset and fills the
// missing chroma by bilinear interpolation of the four neighbouring samples);
// section 3.7 (K-frames: down every column of the quantised lowpass, each
// element becomes its difference with the element above).
//
// The bodies are __host__ __device__ so that their indexing can be run on
// the CPU against bounds-checked buffers; the kernels in ct_color.hip call
// them once per thread. All offsets are 32-bit: the host rejects calls whose
// buffers exceed 2^31 elements.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ct {
namespace color {

constexpr int kPix = 4;              // consecutive pixels per thread
constexpr float kChromaOffset = 127.0f;
constexpr int kDiffRows = 32;        // lowpass rows loaded before any store

// Colour planes of a batch: Y at full size [B][H][W], chroma [B][Hc][Wc] with
// Hc = ceil(H / n), Wc = ceil(W / n).
struct Frame {
    int H, W, n, Hc, Wc;
    uint32_t P;   // B * H * W pixels
};

// Position of a pixel of the flattened batch, advanced one pixel at a time
// without divisions: (plane, row, column), the row and column modulo n, and
// the chroma sample row and column at or before it.
struct Pos {
    uint32_t b, y, x, ym, xm, i, j;

    __host__ __device__ void init(uint32_t p, const Frame& f) {
        const uint32_t row = p / uint32_t(f.W);
        x = p - row * uint32_t(f.W);
        b = row / uint32_t(f.H);
        y = row - b * uint32_t(f.H);
        i = y / uint32_t(f.n);
        ym = y - i * uint32_t(f.n);
        j = x / uint32_t(f.n);
        xm = x - j * uint32_t(f.n);
    }
    __host__ __device__ void next(const Frame& f) {
        ++x;
        if (++xm == uint32_t(f.n)) {
            xm = 0;
            ++j;
        }
        if (x == uint32_t(f.W)) {
            x = xm = j = 0;
            ++y;
            if (++ym == uint32_t(f.n)) {
                ym = 0;
                ++i;
            }
            if (y == uint32_t(f.H)) {
                y = ym = i = 0;
                ++b;
            }
        }
    }
    __host__ __device__ uint32_t sample(const Frame& f, uint32_t si, uint32_t sj) const {
        return (b * uint32_t(f.Hc) + si) * uint32_t(f.Wc) + sj;
    }
};

// Equations (1)-(3) and the +127 chroma offset. Every product and sum of
// 8-bit values here is a multiple of 1/4 below 2^10, so float32 is exact.
__host__ __device__ inline float luma(float r, float g, float b) {
    return (0.25f * r + 0.5f * g) + 0.25f * b;
}
__host__ __device__ inline float chroma_o(float r, float b) {
    return (0.5f * r - 0.5f * b) + kChromaOffset;
}
__host__ __device__ inline float chroma_g(float r, float g, float b) {
    return (-0.25f * r + 0.5f * g - 0.25f * b) + kChromaOffset;
}

// Converts `cnt` pixels starting at p0 (r, g, b already unpacked): Y for
// each, and Co, Cg where the pixel is a kept chroma sample. A full group
// stores Y as one float4 (`y` 16-byte aligned).
__host__ __device__ inline void ycocg_from(uint32_t p0, uint32_t cnt, const float* r,
                                           const float* g, const float* b,
                                           float* __restrict__ y, float* __restrict__ co,
                                           float* __restrict__ cg, const Frame& f) {
    if (cnt == kPix) {
        float4 v;
        v.x = luma(r[0], g[0], b[0]);
        v.y = luma(r[1], g[1], b[1]);
        v.z = luma(r[2], g[2], b[2]);
        v.w = luma(r[3], g[3], b[3]);
        *reinterpret_cast<float4*>(y + p0) = v;
    } else {
        for (uint32_t k = 0; k < cnt; ++k) y[p0 + k] = luma(r[k], g[k], b[k]);
    }
    Pos pos;
    pos.init(p0, f);
    for (uint32_t k = 0; k < cnt; ++k) {
        if (pos.ym == 0 && pos.xm == 0) {
            const uint32_t s = pos.sample(f, pos.i, pos.j);
            co[s] = chroma_o(r[k], b[k]);
            cg[s] = chroma_g(r[k], g[k], b[k]);
        }
        pos.next(f);
    }
}

// Forward for a full group of thread t whose 12 RGB bytes are the words
// w[0..2] (little endian: R, G, B of pixel 0 in the low bytes of w[0]).
__host__ __device__ inline void rgb_to_ycocg_words(uint32_t t, const uint32_t* w,
                                                   float* __restrict__ y, float* __restrict__ co,
                                                   float* __restrict__ cg, const Frame& f) {
    float r[kPix], g[kPix], b[kPix];
    for (int k = 0; k < kPix; ++k) {
        const int q0 = 3 * k, q1 = 3 * k + 1, q2 = 3 * k + 2;
        r[k] = float((w[q0 >> 2] >> (8 * (q0 & 3))) & 255);
        g[k] = float((w[q1 >> 2] >> (8 * (q1 & 3))) & 255);
        b[k] = float((w[q2 >> 2] >> (8 * (q2 & 3))) & 255);
    }
    ycocg_from(t * kPix, kPix, r, g, b, y, co, cg, f);
}

// Forward: thread t converts pixels 4t .. 4t+3 of the batch. `rgb` is
// 4-byte aligned; a full group reads three words.
__host__ __device__ inline void rgb_to_ycocg(uint32_t t, const uint8_t* __restrict__ rgb,
                                             float* __restrict__ y, float* __restrict__ co,
                                             float* __restrict__ cg, const Frame& f) {
    const uint32_t p0 = t * kPix;
    if (p0 >= f.P) return;
    const uint32_t cnt = f.P - p0 < uint32_t(kPix) ? f.P - p0 : uint32_t(kPix);
    if (cnt == kPix) {
        const uint32_t* src = reinterpret_cast<const uint32_t*>(rgb + 3 * p0);
        const uint32_t w[3] = {src[0], src[1], src[2]};
        rgb_to_ycocg_words(t, w, y, co, cg, f);
        return;
    }
    float r[kPix], g[kPix], b[kPix];
    for (uint32_t k = 0; k < cnt; ++k) {
        r[k] = float(rgb[3 * (p0 + k)]);
        g[k] = float(rgb[3 * (p0 + k) + 1]);
        b[k] = float(rgb[3 * (p0 + k) + 2]);
    }
    ycocg_from(p0, cnt, r, g, b, y, co, cg, f);
}

// Float at a byte offset from a uniform base (32-bit offsets let the
// compiler keep the base in scalar registers).
__host__ __device__ inline float ld_f(const float* base, uint32_t byte_off) {
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + byte_off);
}

// Bilinear mixing: between the two sample rows first, then between the two
// sample columns, then the offset removed.
__host__ __device__ inline float vmix(float top, float bottom, float fy) {
    return (1.0f - fy) * top + fy * bottom;
}
__host__ __device__ inline float hmix(float left, float right, float fx) {
    return ((1.0f - fx) * left + fx * right) - kChromaOffset;
}

// Bilinear value at the current pixel of one chroma plane, offset removed.
__host__ __device__ inline float upsample_at(const float* __restrict__ c, const Pos& pos,
                                             const Frame& f, float fy, float fx) {
    const uint32_t i1 = pos.i + 1 < uint32_t(f.Hc) ? pos.i + 1 : pos.i;
    const uint32_t j1 = pos.j + 1 < uint32_t(f.Wc) ? pos.j + 1 : pos.j;
    const float c00 = c[pos.sample(f, pos.i, pos.j)], c01 = c[pos.sample(f, pos.i, j1)];
    const float c10 = c[pos.sample(f, i1, pos.j)], c11 = c[pos.sample(f, i1, j1)];
    return hmix(vmix(c00, c10, fy), vmix(c01, c11, fy), fx);
}

// Element `k` of a register window, selected without indexing memory.
template <int K>
__host__ __device__ inline float pick(const float (&v)[K], uint32_t k) {
    float r = v[0];
    for (int q = 1; q < K; ++q) r = k == uint32_t(q) ? v[q] : r;
    return r;
}

// Equations (4)-(6) for pixel k of a group.
__host__ __device__ inline void to_rgb(float* out, int k, float yv, float o, float g) {
    out[3 * k] = (yv + o) - g;
    out[3 * k + 1] = yv + g;
    out[3 * k + 2] = (yv - o) - g;
}

// Chroma columns the inverse loads per group for a factor n: four
// consecutive pixels span at most 4, 3 or 2 sample columns for n = 1, 2 and
// n >= 3, plus the right neighbour of the last.
__host__ __device__ constexpr int window_cols(int n) { return n == 1 ? 5 : n == 2 ? 4 : 3; }

// Inverse: thread t reconstructs pixels 4t .. 4t+3 as float RGB into
// out[0..11] and returns how many it covers (0 past the end). `y` is
// 16-byte aligned; a full group reads one float4.
// `rn` is 1/n rounded to float32: the interpolation weights are (y mod n)/n
// and (x mod n)/n. A full group inside one row (the common case) loads a
// window of K = window_cols(n) chroma columns from the two sample rows, all
// loads before any arithmetic, and mixes each column between the rows once.
// The per-pixel path for the other groups runs the same float32 operations,
// so a pixel's value does not depend on the path.
template <int K>
__host__ __device__ inline uint32_t rgb_group(uint32_t t, const float* __restrict__ y,
                                              const float* __restrict__ co,
                                              const float* __restrict__ cg, const Frame& f,
                                              float rn, float* out /* [3 * kPix] */) {
    const uint32_t p0 = t * kPix;
    if (p0 >= f.P) return 0;
    const uint32_t cnt = f.P - p0 < uint32_t(kPix) ? f.P - p0 : uint32_t(kPix);
    float yv[kPix];
    if (cnt == kPix) {
        const float4 v = *reinterpret_cast<const float4*>(y + p0);
        yv[0] = v.x;
        yv[1] = v.y;
        yv[2] = v.z;
        yv[3] = v.w;
    } else {
        for (uint32_t k = 0; k < uint32_t(kPix); ++k) yv[k] = y[k < cnt ? p0 + k : p0];
    }
    Pos pos;
    pos.init(p0, f);
    if (cnt == kPix && pos.x + (kPix - 1) < uint32_t(f.W)) {
        const uint32_t i1 = pos.i + 1 < uint32_t(f.Hc) ? pos.i + 1 : pos.i;
        const uint32_t row0 = (pos.b * uint32_t(f.Hc) + pos.i) * uint32_t(f.Wc) * 4;
        const uint32_t row1 = (pos.b * uint32_t(f.Hc) + i1) * uint32_t(f.Wc) * 4;
        const uint32_t jl = uint32_t(f.Wc) - 1;
        float o0[K], o1[K], g0[K], g1[K];
        for (int k = 0; k < K; ++k) {
            const uint32_t cb = 4 * (pos.j + k < jl ? pos.j + k : jl);
            o0[k] = ld_f(co, row0 + cb);
            o1[k] = ld_f(co, row1 + cb);
            g0[k] = ld_f(cg, row0 + cb);
            g1[k] = ld_f(cg, row1 + cb);
        }
        const float fy = float(pos.ym) * rn;
        float ov[K], gv[K];
        for (int k = 0; k < K; ++k) {
            ov[k] = vmix(o0[k], o1[k], fy);
            gv[k] = vmix(g0[k], g1[k], fy);
        }
        uint32_t xm = pos.xm, jr = 0;
        for (int k = 0; k < kPix; ++k) {
            if (K == window_cols(1)) {   // n = 1: pixel k sits on sample column k, weight 0
                xm = 0;
                jr = uint32_t(k);
            }
            const float fx = float(xm) * rn;
            to_rgb(out, k, yv[k], hmix(pick(ov, jr), pick(ov, jr + 1), fx),
                   hmix(pick(gv, jr), pick(gv, jr + 1), fx));
            if (++xm == uint32_t(f.n)) {
                xm = 0;
                ++jr;
            }
        }
    } else {
        for (uint32_t k = 0; k < uint32_t(kPix); ++k) {
            const float fy = float(pos.ym) * rn, fx = float(pos.xm) * rn;
            to_rgb(out, k, yv[k], upsample_at(co, pos, f, fy, fx),
                   upsample_at(cg, pos, f, fy, fx));
            if (k + 1 < cnt) pos.next(f);
        }
    }
    return cnt;
}

// Stores the `cnt` pixels of thread t's group (three float4 for a full
// group; `rgb` 16-byte aligned).
__host__ __device__ inline void store_rgb(uint32_t t, uint32_t cnt, const float* out,
                                          float* __restrict__ rgb) {
    const size_t o = 3 * size_t(t) * kPix;
    if (cnt == kPix) {
        float4* o4 = reinterpret_cast<float4*>(rgb + o);
        o4[0] = make_float4(out[0], out[1], out[2], out[3]);
        o4[1] = make_float4(out[4], out[5], out[6], out[7]);
        o4[2] = make_float4(out[8], out[9], out[10], out[11]);
    } else {
        for (uint32_t k = 0; k < 3 * cnt; ++k) rgb[o + k] = out[k];
    }
}

template <int K>
__host__ __device__ inline void ycocg_to_rgb(uint32_t t, const float* __restrict__ y,
                                             const float* __restrict__ co,
                                             const float* __restrict__ cg, float* __restrict__ rgb,
                                             const Frame& f, float rn) {
    float out[3 * kPix];
    const uint32_t cnt = rgb_group<K>(t, y, co, cg, f, rn, out);
    if (cnt) store_rgb(t, cnt, out, rgb);
}

// K-frame lowpass filtering in place, thread t owning one column of one
// plane's lowpass (rows x cols, row major, planes `plane` elements apart).
// Forward: row 0 kept, row i becomes x[i] - x[i-1] of the input. Inverse:
// running sums down the column. Both wrap modulo 2^16, so the inverse
// restores any int16 input exactly. Each thread reads a chunk of rows before
// it writes any, and touches only its own column.
__host__ __device__ inline void lowpass_diff(uint32_t t, int16_t* idx, uint32_t plane, int rows,
                                             int cols, int batch, bool inverse) {
    if (t >= uint32_t(batch) * uint32_t(cols)) return;
    const uint32_t b = t / uint32_t(cols), c = t - b * uint32_t(cols);
    int16_t* p = idx + b * plane + c;
    int carry = 0;
    for (int i0 = 0; i0 < rows; i0 += kDiffRows) {
        int v[kDiffRows];
        for (int k = 0; k < kDiffRows; ++k)
            if (i0 + k < rows) v[k] = p[uint32_t(i0 + k) * uint32_t(cols)];
        for (int k = 0; k < kDiffRows; ++k) {
            const int i = i0 + k;
            if (i >= rows) break;
            if (i == 0) {
                carry = v[k];
                continue;
            }
            int16_t outv;
            if (inverse) {
                carry = int16_t(carry + v[k]);
                outv = int16_t(carry);
            } else {
                outv = int16_t(v[k] - carry);
                carry = v[k];
            }
            p[uint32_t(i) * uint32_t(cols)] = outv;
        }
    }
}

}  // namespace color
}  // namespace ct

// Quantiser stages (device functions), shared by the quantiser kernels, the
// group kernels of the batched form and the quantising transform stages. The float32 operation order is part of the
// contract (ct.h, ct_quantize): every function body disables FMA contraction
// (the _rn helpers are plain operators in this toolchain configuration).
//
// Paper section 3.4 (lowpass normalised to [0, 255], restored at the
// decoder), section 3.5 (division by QPH / QPL), section 3.6 (rounding to the
// nearest integer).
#pragma once

#include <math.h>

#include "ct_internal.h"
#include "ct_kernels.h"

namespace ct {
namespace qstage {

constexpr int CHUNK = 4096;     // coefficients per quantiser tile

template <int NT>
__device__ __forceinline__ void block_minmax(float& mn, float& mx, float* red) {
    for (int o = 32; o > 0; o >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, o, 64));
        mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        red[2 * w] = mn;
        red[2 * w + 1] = mx;
    }
    __syncthreads();
    mn = red[0];
    mx = red[1];
    for (int i = 1; i < NT / 64; ++i) {
        mn = fminf(mn, red[2 * i]);
        mx = fmaxf(mx, red[2 * i + 1]);
    }
    __syncthreads();
}

// round(v) with halves away from zero, saturated to int16, NaN -> 0, with
// selects only (no branches): trunc(v + copysign(0.5 - 2^-25, v)) equals
// roundf(v) for every float (checked over all 2^32 bit patterns against the
// branching form); the largest float below one half keeps a value just
// under k + 1/2 from rounding up in the addition.
__host__ __device__ __forceinline__ int16_t to_index(float v) {
    const float r = __builtin_truncf(v + __builtin_copysignf(0x1.fffffep-2f, v));   // one rounding
    const float c = __builtin_fminf(__builtin_fmaxf(r, -32768.f), 32767.f);
    return v == v ? (int16_t)(int)c : (int16_t)0;
}

// Steps in [2^-20, 2^20] take the index through the reciprocal below; others
// the correctly rounded division.
__host__ __device__ inline bool fast_step(float b) { return b >= 0x1p-20f && b <= 0x1p20f; }

// to_index(a / b rounded to nearest) for a step b with fast_step(b) and
// r = 1 / b rounded to nearest: the quotient a r corrected twice by its
// residual a - b q, each residual exact in one FMA (Markstein's correction
// of a reciprocal-based quotient). Wherever the index depends on it this is
// the correctly rounded quotient; where |a r| >= 2^24 the index saturates
// either way and a r is kept (no overflow in the residuals). Checked against
// the division for every float a and 1,831 steps: the integers and halves to
// 128, the powers of two, mantissas of all ones and near them, and 1,200
// log-uniform steps over the range.
__host__ __device__ __forceinline__ int16_t quant_index(float a, float b, float r) {
    const float q0 = a * r;   // one rounding (no contraction in this file's builds)
    const float q1 = __builtin_fmaf(__builtin_fmaf(-b, q0, a), r, q0);
    const float q2 = __builtin_fmaf(__builtin_fmaf(-b, q1, a), r, q1);
    return to_index(__builtin_fabsf(q0) < 0x1p24f ? q2 : q0);
}

// The quantiser's index of a / b; `fast` (uniform across the wave) says that
// fast_step(b) holds and r is 1 / b rounded to nearest.
__device__ __forceinline__ int16_t index_of(float a, float b, float r, bool fast) {
    return fast ? quant_index(a, b, r) : to_index(__fdiv_rn(a, b));
}

__device__ __forceinline__ int find_subband(const QuantArgs& A, int64_t e) {
    int lo = 0, hi = A.nsub - 1;           // largest s with sub_off[s] <= e
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.sub_off[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int partial_tiles(const QuantArgs& A, int batch) { return A.nparts * batch; }
__device__ __forceinline__ int chunk_tiles(const QuantArgs& A, int batch) {
    return int((A.nq + CHUNK - 1) / CHUNK) * batch;
}

// Pass 1: (min, max) of one block of one plane's lowpass.
template <int NT>
__device__ void lowpass_partial(const QuantArgs& A, int tile, float* red) {
#pragma clang fp contract(off)
    const int b = tile / A.nparts, p = tile - b * A.nparts;
    const int64_t per = (A.low_n + A.nparts - 1) / A.nparts;
    const int64_t lo = p * per;
    const int64_t hi = lo + per < A.low_n ? lo + per : A.low_n;
    const float* c = A.coeffs + b * A.in_plane;
    float mn = INFINITY, mx = -INFINITY;
    for (int64_t e = lo + threadIdx.x; e < hi; e += NT) {
        const float v = c[e];
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
    }
    block_minmax<NT>(mn, mx, red);
    if (threadIdx.x == 0) {
        A.partials[(int64_t(b) * kMaxPart + p) * 2 + 0] = mn;
        A.partials[(int64_t(b) * kMaxPart + p) * 2 + 1] = mx;
    }
}

// Pass 2: indices of one chunk of CHUNK coefficients of one plane.
template <int NT>
__device__ void quantize(const QuantArgs& A, int tile, float* red) {
#pragma clang fp contract(off)
    constexpr int ITEMS = CHUNK / NT;
    const int nch = int((A.nq + CHUNK - 1) / CHUNK);
    const int b = tile / nch;
    const int64_t e0 = int64_t(tile - b * nch) * CHUNK;
    float mn = 0.f, mx = 0.f, sc = 0.f;
    if (e0 < A.low_n) {
        float pmn = INFINITY, pmx = -INFINITY;
        for (int p = threadIdx.x; p < A.nparts; p += NT) {
            pmn = fminf(pmn, A.partials[(int64_t(b) * kMaxPart + p) * 2 + 0]);
            pmx = fmaxf(pmx, A.partials[(int64_t(b) * kMaxPart + p) * 2 + 1]);
        }
        block_minmax<NT>(pmn, pmx, red);
        mn = pmn;
        mx = pmx;
        sc = (mx == mn) ? 0.f : __fdiv_rn(255.f, __fsub_rn(mx, mn));
        if (e0 == 0 && threadIdx.x == 0) {
            A.side[2 * b + 0] = mn;
            A.side[2 * b + 1] = mx;
        }
    }
    const float* c = A.coeffs + b * A.in_plane;
    int16_t* q = A.idx + b * A.ncoef;
    const float* steps = A.steps + int64_t(b) * A.steps_stride;
    const int64_t e_end = e0 + CHUNK < A.nq ? e0 + CHUNK : A.nq;
    const int s0 = find_subband(A, e0);
    if (A.vec8 && A.sub_off[s0 + 1] >= e_end) {
        // the whole chunk lies in one subband: 8 consecutive coefficients per
        // thread, 32-byte loads and a 16-byte store
        constexpr int IT = (CHUNK / 8 + NT - 1) / NT;
        const float step = steps[s0];
        const bool fast = __builtin_amdgcn_readfirstlane(int(fast_step(step))) != 0;
        const float rstep = fast ? __fdiv_rn(1.f, step) : 1.f;
        float4 xa[IT], xb[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int64_t e = e0 + 8 * (threadIdx.x + it * NT);
            if (e < e_end) {
                xa[it] = *reinterpret_cast<const float4*>(c + e);
                xb[it] = *reinterpret_cast<const float4*>(c + e + 4);
            }
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int64_t e = e0 + 8 * (threadIdx.x + it * NT);
            if (e >= e_end) break;
            const float x[8] = {xa[it].x, xa[it].y, xa[it].z, xa[it].w,
                                xb[it].x, xb[it].y, xb[it].z, xb[it].w};
            uint32_t w[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                uint32_t pair[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const float xv = x[2 * h + u];
                    const float a = s0 == 0 ? __fmul_rn(__fsub_rn(xv, mn), sc) : xv;
                    pair[u] = uint32_t(uint16_t(index_of(a, step, rstep, fast)));
                }
                w[h] = pair[0] | (pair[1] << 16);
            }
            *reinterpret_cast<uint4*>(q + e) = make_uint4(w[0], w[1], w[2], w[3]);
        }
        return;
    }
    const int64_t e_first = e0 + threadIdx.x;
    if (e_first >= A.nq) return;
    float xs[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int64_t e = e_first + int64_t(it) * NT;
        xs[it] = e < A.nq ? c[e] : 0.f;
    }
    int s = find_subband(A, e_first);
    int64_t next = A.sub_off[s + 1];
    float step = steps[s];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int64_t e = e_first + int64_t(it) * NT;
        if (e >= A.nq) break;
        while (e >= next) {
            ++s;
            next = A.sub_off[s + 1];
            step = steps[s];
        }
        float v;
        if (s == 0)
            v = __fdiv_rn(__fmul_rn(__fsub_rn(xs[it], mn), sc), step);
        else
            v = __fdiv_rn(xs[it], step);
        q[e] = to_index(v);
    }
}

// Dequantise one chunk.
template <int NT>
__device__ void dequantize(const QuantArgs& A, int tile) {
#pragma clang fp contract(off)
    constexpr int ITEMS = CHUNK / NT;
    const int nch = int((A.ncoef + CHUNK - 1) / CHUNK);
    const int b = tile / nch;
    const int64_t e0 = int64_t(tile - b * nch) * CHUNK;
    const float mn = A.side[2 * b + 0], mx = A.side[2 * b + 1];
    const float r = __fdiv_rn(__fsub_rn(mx, mn), 255.f);
    const int16_t* q = A.idx_in + b * A.ncoef;
    float* out = A.coeffs_out + b * A.ncoef;
    const float* steps = A.steps + int64_t(b) * A.steps_stride;
    const int64_t e_end = e0 + CHUNK < A.ncoef ? e0 + CHUNK : A.ncoef;
    const int s0 = find_subband(A, e0);
    if (A.vec8 && A.sub_off[s0 + 1] >= e_end) {
        // one subband: a 16-byte load and two 16-byte stores per thread
        constexpr int IT = (CHUNK / 8 + NT - 1) / NT;
        const float step = steps[s0];
        uint4 qa[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int64_t e = e0 + 8 * (threadIdx.x + it * NT);
            if (e < e_end) qa[it] = *reinterpret_cast<const uint4*>(q + e);
        }
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int64_t e = e0 + 8 * (threadIdx.x + it * NT);
            if (e >= e_end) break;
            const uint32_t w[4] = {qa[it].x, qa[it].y, qa[it].z, qa[it].w};
            float y[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int16_t qi = int16_t(uint16_t(w[u >> 1] >> (16 * (u & 1))));
                const float v = __fmul_rn((float)qi, step);
                y[u] = s0 == 0 ? __fadd_rn(mn, __fmul_rn(v, r)) : v;
            }
            *reinterpret_cast<float4*>(out + e) = make_float4(y[0], y[1], y[2], y[3]);
            *reinterpret_cast<float4*>(out + e + 4) = make_float4(y[4], y[5], y[6], y[7]);
        }
        return;
    }
    const int64_t e_first = e0 + threadIdx.x;
    if (e_first >= A.ncoef) return;
    int16_t qs[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int64_t e = e_first + int64_t(it) * NT;
        qs[it] = e < A.ncoef ? q[e] : int16_t(0);
    }
    int s = find_subband(A, e_first);
    int64_t next = A.sub_off[s + 1];
    float step = steps[s];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int64_t e = e_first + int64_t(it) * NT;
        if (e >= A.ncoef) break;
        while (e >= next) {
            ++s;
            next = A.sub_off[s + 1];
            step = steps[s];
        }
        const float w = __fmul_rn((float)qs[it], step);
        out[e] = (s == 0) ? __fadd_rn(mn, __fmul_rn(w, r)) : w;
    }
}

}  // namespace qstage
}  // namespace ct

// Device helpers shared by the LP and DFB kernels: periodic indexing, the
// separable LP filter passes on LDS tiles, and the lifting steps of DFB tree
// levels 1 and 2.
#pragma once

#include "ct_kernels.h"

namespace ct {
namespace dev {

__device__ __forceinline__ int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

// i mod n (non-negative) with a float reciprocal inv = 1/n instead of an
// integer division: the float quotient is off by at most one for |i| < 2^22,
// which the two corrections absorb.
__device__ __forceinline__ int fwrap(int i, int n, float inv) {
    int r = i - int(floorf(float(i) * inv)) * n;
    if (r < 0) r += n;
    if (r >= n) r -= n;
    return r;
}

// ---------------------------------------------------------------- LP passes
// A tile stores its full-resolution input `in` with the lowpass grid aligned
// so that lowpass sample t (local) sits over input column 4 + 2t, and lowpass
// row s over input row 4 + 2s.

// hf[r][t] = sum_k lo[k] in[r][4 + 2t +- k], rows [0, NR), lowpass cols [0, NC).
template <int LO_R, int NR, int NC, int IN_LD, int HF_LD, int NT>
__device__ __forceinline__ void rows_lo(const float* in, float* hf, const Taps5& lo) {
    for (int idx = threadIdx.x; idx < NR * NC; idx += NT) {
        const int r = idx / NC, t = idx - r * NC;
        const float* row = in + r * IN_LD + 4 + 2 * t;
        float acc = lo.t[0] * row[0];
#pragma unroll
        for (int k = 1; k <= LO_R; ++k) acc += lo.t[k] * (row[-k] + row[k]);
        hf[r * HF_LD + t] = acc;
    }
}

// sum_k lo[k] hf[4 + 2s +- k][t]: the column pass at lowpass row s.
template <int LO_R, int HF_LD>
__device__ __forceinline__ float cols_lo(const float* hf, const Taps5& lo, int s, int t) {
    const float* col = hf + (4 + 2 * s) * HF_LD + t;
    float acc = lo.t[0] * col[0];
#pragma unroll
    for (int k = 1; k <= LO_R; ++k) acc += lo.t[k] * (col[-k * HF_LD] + col[k * HF_LD]);
    return acc;
}

// uh[s][j] = sum_m up[j + 4 - 2m] c[s][m] for output columns j in [0, NJ):
// polyphase upsampling along rows.
template <int UP_R, int NS, int NJ, int C_LD, int UH_LD, int NT>
__device__ __forceinline__ void rows_up(const float* c, float* uh, const Taps5& up) {
    for (int idx = threadIdx.x; idx < NS * NJ; idx += NT) {
        const int r = idx / NJ, j = idx - r * NJ;
        const int p = j & 1, base = (j >> 1) + 2;
        const float* cr = c + r * C_LD;
        float acc = 0.f;
#pragma unroll
        for (int i = -2; i <= 2; ++i) {
            const int tau = p + 2 * i;
            const int at = tau < 0 ? -tau : tau;
            if (at <= UP_R) acc += up.t[at] * cr[base - i];
        }
        uh[r * UH_LD + j] = acc;
    }
}

// Column upsampling at output row i, column j.
template <int UP_R, int UH_LD>
__device__ __forceinline__ float cols_up(const float* uh, const Taps5& up, int i, int j) {
    const int p = i & 1, base = (i >> 1) + 2;
    float acc = 0.f;
#pragma unroll
    for (int ii = -2; ii <= 2; ++ii) {
        const int tau = p + 2 * ii;
        const int at = tau < 0 ? -tau : tau;
        if (at <= UP_R) acc += up.t[at] * uh[(base - ii) * UH_LD + j];
    }
    return acc;
}

// ---------------------------------------------------------------- DFB 1-2
// Lifting step of DFB tree level 1 on a square tile of side N (row stride LD)
// over rows/cols [m, N - m): points with (r + c) & 1 == par are updated from
// their horizontal (+) and vertical (-) neighbours.
template <int N, int LD, int NT>
__device__ __forceinline__ void step_cross(float* T, int par, float coef, int m) {
    const int span = N - 2 * m;
    const int half = span / 2;
    // (row, half-column) of this thread's first point and the per-iteration
    // advance, so the loop needs no division per point
    const int q = NT / half, rmd = NT - q * half;
    int rr = threadIdx.x / half, j = threadIdx.x - rr * half;
    while (rr < span) {
        const int r = m + rr;
        const int c = m + 2 * j + ((r + m + par) & 1);
        float* p = T + r * LD + c;
        *p += coef * ((p[1] + p[-1]) - (p[LD] + p[-LD]));
        rr += q;
        j += rmd;
        if (j >= half) {
            j -= half;
            ++rr;
        }
    }
}

// Lifting step of DFB tree level 2: points with c & 1 == par are updated from
// their anti-diagonal (+) and diagonal (-) neighbours.
template <int N, int LD, int NT>
__device__ __forceinline__ void step_diag(float* T, int par, float coef, int m) {
    const int span = N - 2 * m;
    const int half = span / 2;
    const int q = NT / half, rmd = NT - q * half;
    int rr = threadIdx.x / half, j = threadIdx.x - rr * half;
    const int c0 = m + ((m + par) & 1);
    while (rr < span) {
        float* p = T + (m + rr) * LD + c0 + 2 * j;
        *p += coef * ((p[-LD + 1] + p[LD - 1]) - (p[LD + 1] + p[-LD - 1]));
        rr += q;
        j += rmd;
        if (j >= half) {
            j -= half;
            ++rr;
        }
    }
}

}  // namespace dev
}  // namespace ct

// Quantiser and dequantiser kernels for gfx950.
//
// Paper section 3.4 (lowpass normalised to [0, 255] and restored at the
// decoder), section 3.5 (division by QPH / QPL, then rounding to an
// integer), section 3.6 (rounding to the nearest integer).
//
// Per plane: mn, mx = min, max of the lowpass. Then, in IEEE float32 with
// every operation correctly rounded and in this order (this translation unit
// is built without FMA contraction):
//   lowpass      d = mx - mn; s = 255 / d (0 if mx == mn); t = c - mn;
//                u = t * s; v = u / step[0]
//   directional  v = c / step[i]
//   q = round half away from zero (roundf), saturated to int16, NaN -> 0.
// Dequantise: c = q * step[i]; lowpass c = mn + (q * step[0]) * ((mx - mn) / 255).
//
// The lowpass min/max is a two-pass reduction without atomics: pass 1 writes
// one (min, max) partial per block of the lowpass; the quantise pass reduces
// the partials of its plane with wavefront shuffles before use, so the
// result does not depend on scheduling.
#include <math.h>

#include "ct_internal.h"
#include "ct_kernels.h"

namespace ct {
namespace {

constexpr int NT = 256;
constexpr int ITEMS = 16;                 // elements per thread
constexpr int CHUNK = NT * ITEMS;         // elements per block

__device__ __forceinline__ float wave_min(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide min and max; every thread gets the result.
__device__ void block_minmax(float& mn, float& mx) {
    __shared__ float smn[NT / 64], smx[NT / 64];
    mn = wave_min(mn);
    mx = wave_max(mx);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        smn[w] = mn;
        smx[w] = mx;
    }
    __syncthreads();
    mn = smn[0];
    mx = smx[0];
    for (int i = 1; i < NT / 64; ++i) {
        mn = fminf(mn, smn[i]);
        mx = fmaxf(mx, smx[i]);
    }
}

__global__ __launch_bounds__(NT) void lowpass_partial_kernel(QuantArgs A) {
    const int b = blockIdx.y, p = blockIdx.x;
    const int64_t per = (A.low_n + A.nparts - 1) / A.nparts;
    const int64_t lo = p * per;
    const int64_t hi = lo + per < A.low_n ? lo + per : A.low_n;
    const float* c = A.coeffs + b * A.ncoef;
    float mn = INFINITY, mx = -INFINITY;
    for (int64_t e = lo + threadIdx.x; e < hi; e += NT) {
        const float v = c[e];
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
    }
    block_minmax(mn, mx);
    if (threadIdx.x == 0) {
        A.partials[(int64_t(b) * kMaxPart + p) * 2 + 0] = mn;
        A.partials[(int64_t(b) * kMaxPart + p) * 2 + 1] = mx;
    }
}

__device__ __forceinline__ int16_t to_index(float v) {
    const float r = roundf(v);            // halves away from zero
    if (!(r == r)) return 0;              // NaN
    if (r >= 32767.f) return 32767;
    if (r <= -32768.f) return -32768;
    return (int16_t)(int)r;
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

__global__ __launch_bounds__(NT) void quantize_kernel(QuantArgs A) {
    const int b = blockIdx.y;
    const int64_t e0 = int64_t(blockIdx.x) * CHUNK;
    float mn = 0.f, mx = 0.f, sc = 0.f;
    if (e0 < A.low_n) {
        float pmn = INFINITY, pmx = -INFINITY;
        for (int p = threadIdx.x; p < A.nparts; p += NT) {
            pmn = fminf(pmn, A.partials[(int64_t(b) * kMaxPart + p) * 2 + 0]);
            pmx = fmaxf(pmx, A.partials[(int64_t(b) * kMaxPart + p) * 2 + 1]);
        }
        block_minmax(pmn, pmx);
        mn = pmn;
        mx = pmx;
        sc = (mx == mn) ? 0.f : __fdiv_rn(255.f, __fsub_rn(mx, mn));
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            A.side[2 * b + 0] = mn;
            A.side[2 * b + 1] = mx;
        }
    }
    const float* c = A.coeffs + b * A.ncoef;
    int16_t* q = A.idx + b * A.ncoef;
    const float* steps = A.steps + int64_t(b) * A.steps_stride;
    const int64_t e_first = e0 + threadIdx.x;
    if (e_first >= A.ncoef) return;
    // issue every load of this thread before any arithmetic (memory-level parallelism)
    float xs[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int64_t e = e_first + int64_t(it) * NT;
        xs[it] = e < A.ncoef ? c[e] : 0.f;
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
        float v;
        if (s == 0)
            v = __fdiv_rn(__fmul_rn(__fsub_rn(xs[it], mn), sc), step);
        else
            v = __fdiv_rn(xs[it], step);
        q[e] = to_index(v);
    }
}

__global__ __launch_bounds__(NT) void dequantize_kernel(QuantArgs A) {
    const int b = blockIdx.y;
    const int64_t e0 = int64_t(blockIdx.x) * CHUNK;
    const float mn = A.side[2 * b + 0], mx = A.side[2 * b + 1];
    const float r = __fdiv_rn(__fsub_rn(mx, mn), 255.f);
    const int16_t* q = A.idx_in + b * A.ncoef;
    float* out = A.coeffs_out + b * A.ncoef;
    const float* steps = A.steps + int64_t(b) * A.steps_stride;
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

}  // namespace

hipError_t launch_lowpass_partial(const QuantArgs& a, int batch, hipStream_t st) {
    lowpass_partial_kernel<<<dim3(a.nparts, batch), NT, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_quantize(const QuantArgs& a, int batch, hipStream_t st) {
    const unsigned nblk = unsigned((a.ncoef + CHUNK - 1) / CHUNK);
    quantize_kernel<<<dim3(nblk, batch), NT, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_dequantize(const QuantArgs& a, int batch, hipStream_t st) {
    const unsigned nblk = unsigned((a.ncoef + CHUNK - 1) / CHUNK);
    dequantize_kernel<<<dim3(nblk, batch), NT, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace ct

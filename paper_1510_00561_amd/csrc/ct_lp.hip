// Laplacian pyramid kernels for gfx950.
//
// Paper section 2.1: each LP level splits its input into a half-resolution
// lowpass and a full-resolution bandpass; section 3.10: the convolutions are
// periodic (FFT based). Reading: unit-DC 9-7 filters and dual-frame
// reconstruction.
//
//   analysis   c = down2(lo * x)          d = x - up * up2(c)
//   synthesis  c' = c - down2(lo * d)     x = d + up * up2(c')
//
// Forward uses (lo, up) = (hbar, gbar); the transposes use the same kernels
// with the filters swapped. Each 256-thread workgroup produces a 32 x 64 tile
// of the full-resolution output. It stages the input tile plus an 8-pixel
// halo in LDS with periodic wrap (and, on the first level, mirror or zero
// padding past the real frame), filters rows then columns on the decimated
// grid, and upsamples through the polyphase taps of `up`. Every global load
// and store runs along rows, so a wavefront touches contiguous memory.
#include "ct_kernels.h"

namespace ct {
namespace {

constexpr int TH = 32, TW = 64, HALO = 8;
constexpr int IN_R = TH + 2 * HALO;      // 48
constexpr int IN_C = TW + 2 * HALO;      // 80
constexpr int IN_LD = IN_C + 1;
constexpr int CR = TH / 2 + 4;           // 20 lowpass rows (halo 2)
constexpr int CCOL = TW / 2 + 4;         // 36 lowpass cols (halo 2)
constexpr int C_LD = CCOL + 1;
constexpr int UH_LD = TW + 1;
constexpr int NT = 256;

__device__ __forceinline__ int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

struct LpSmem {
    float in[IN_R][IN_LD];    // x (analysis) or d (synthesis), with halo
    float hf[IN_R][C_LD];     // rows filtered by lo and decimated
    float c[CR][C_LD];        // lowpass tile (c, or c' in synthesis)
    float uh[CR][UH_LD];      // lowpass upsampled and filtered along rows
};

// hf[r][t] = sum_k lo[k] in[r][4 + 2t - k]   (all rows)
template <int LO_R>
__device__ __forceinline__ void rows_lo(LpSmem& s, const Taps5& lo) {
    for (int idx = threadIdx.x; idx < IN_R * CCOL; idx += NT) {
        const int r = idx / CCOL, t = idx - r * CCOL;
        const int cc = 4 + 2 * t;
        float acc = lo.t[0] * s.in[r][cc];
#pragma unroll
        for (int k = 1; k <= LO_R; ++k) acc += lo.t[k] * (s.in[r][cc - k] + s.in[r][cc + k]);
        s.hf[r][t] = acc;
    }
}

// column pass of lo on hf at lowpass row s: sum_k lo[k] hf[4 + 2s - k][t]
template <int LO_R>
__device__ __forceinline__ float cols_lo(const LpSmem& s, const Taps5& lo, int row, int t) {
    const int rc = 4 + 2 * row;
    float acc = lo.t[0] * s.hf[rc][t];
#pragma unroll
    for (int k = 1; k <= LO_R; ++k) acc += lo.t[k] * (s.hf[rc - k][t] + s.hf[rc + k][t]);
    return acc;
}

// uh[s][j] = sum_m up[j + 4 - 2m] c[s][m]  (polyphase upsampling along rows)
template <int UP_R>
__device__ __forceinline__ void rows_up(LpSmem& s, const Taps5& up) {
    for (int idx = threadIdx.x; idx < CR * TW; idx += NT) {
        const int r = idx / TW, j = idx - r * TW;
        const int p = j & 1, base = (j >> 1) + 2;
        float acc = 0.f;
#pragma unroll
        for (int i = -2; i <= 2; ++i) {
            const int tau = p + 2 * i;
            const int at = tau < 0 ? -tau : tau;
            if (at <= UP_R) acc += up.t[at] * s.c[r][base - i];
        }
        s.uh[r][j] = acc;
    }
}

// column upsampling at output row i, column j of the tile
template <int UP_R>
__device__ __forceinline__ float cols_up(const LpSmem& s, const Taps5& up, int i, int j) {
    const int p = i & 1, base = (i >> 1) + 2;
    float acc = 0.f;
#pragma unroll
    for (int ii = -2; ii <= 2; ++ii) {
        const int tau = p + 2 * ii;
        const int at = tau < 0 ? -tau : tau;
        if (at <= UP_R) acc += up.t[at] * s.uh[base - ii][j];
    }
    return acc;
}

template <int LO_R, int UP_R>
__global__ __launch_bounds__(NT) void lp_analysis_kernel(CView src, int src_h, int src_w,
                                                         int pad_mode, int R, int C, View c_out,
                                                         View d_out, Taps5 lo, Taps5 up) {
    __shared__ LpSmem s;
    const int gx = (C + TW - 1) / TW, gy = (R + TH - 1) / TH;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = L % gx, ty = (L / gx) % gy, b = L / (gx * gy);
    const int n0 = ty * TH, m0 = tx * TW;
    const float* sp = src.p + b * src.plane;
    for (int idx = threadIdx.x; idx < IN_R * IN_C; idx += NT) {
        const int r = idx / IN_C, c = idx - r * IN_C;
        int gr = wrap(n0 - HALO + r, R), gc = wrap(m0 - HALO + c, C);
        float v;
        if (pad_mode == kPadReflect) {
            if (gr >= src_h) gr = 2 * src_h - 1 - gr;
            if (gc >= src_w) gc = 2 * src_w - 1 - gc;
            v = sp[int64_t(gr) * src.ld + gc];
        } else if (pad_mode == kPadZero) {
            v = (gr < src_h && gc < src_w) ? sp[int64_t(gr) * src.ld + gc] : 0.f;
        } else {
            v = sp[int64_t(gr) * src.ld + gc];
        }
        s.in[r][c] = v;
    }
    __syncthreads();
    rows_lo<LO_R>(s, lo);
    __syncthreads();
    const int Rh = R >> 1, Ch = C >> 1;
    float* cp = c_out.p + b * c_out.plane;
    for (int idx = threadIdx.x; idx < CR * CCOL; idx += NT) {
        const int r = idx / CCOL, t = idx - r * CCOL;
        const float v = cols_lo<LO_R>(s, lo, r, t);
        s.c[r][t] = v;
        if (r >= 2 && r < CR - 2 && t >= 2 && t < CCOL - 2) {
            const int gr = (n0 >> 1) + r - 2, gc = (m0 >> 1) + t - 2;
            if (gr < Rh && gc < Ch) cp[int64_t(gr) * c_out.ld + gc] = v;
        }
    }
    __syncthreads();
    rows_up<UP_R>(s, up);
    __syncthreads();
    float* dp = d_out.p + b * d_out.plane;
    for (int idx = threadIdx.x; idx < TH * TW; idx += NT) {
        const int i = idx / TW, j = idx - i * TW;
        const int gr = n0 + i, gc = m0 + j;
        if (gr < R && gc < C)
            dp[int64_t(gr) * d_out.ld + gc] = s.in[HALO + i][HALO + j] - cols_up<UP_R>(s, up, i, j);
    }
}

template <int LO_R, int UP_R>
__global__ __launch_bounds__(NT) void lp_synthesis_kernel(CView c_in, CView d_in, int R, int C,
                                                          View x_out, int out_h, int out_w,
                                                          Taps5 lo, Taps5 up) {
    __shared__ LpSmem s;
    const int gx = (C + TW - 1) / TW, gy = (R + TH - 1) / TH;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = L % gx, ty = (L / gx) % gy, b = L / (gx * gy);
    const int n0 = ty * TH, m0 = tx * TW;
    const float* dp = d_in.p + b * d_in.plane;
    for (int idx = threadIdx.x; idx < IN_R * IN_C; idx += NT) {
        const int r = idx / IN_C, c = idx - r * IN_C;
        const int gr = wrap(n0 - HALO + r, R), gc = wrap(m0 - HALO + c, C);
        s.in[r][c] = dp[int64_t(gr) * d_in.ld + gc];
    }
    const int Rh = R >> 1, Ch = C >> 1;
    const float* cp = c_in.p + b * c_in.plane;
    for (int idx = threadIdx.x; idx < CR * CCOL; idx += NT) {
        const int r = idx / CCOL, t = idx - r * CCOL;
        const int gr = wrap((n0 >> 1) - 2 + r, Rh), gc = wrap((m0 >> 1) - 2 + t, Ch);
        s.c[r][t] = cp[int64_t(gr) * c_in.ld + gc];
    }
    __syncthreads();
    rows_lo<LO_R>(s, lo);
    __syncthreads();
    for (int idx = threadIdx.x; idx < CR * CCOL; idx += NT) {
        const int r = idx / CCOL, t = idx - r * CCOL;
        s.c[r][t] -= cols_lo<LO_R>(s, lo, r, t);
    }
    __syncthreads();
    rows_up<UP_R>(s, up);
    __syncthreads();
    float* xp = x_out.p + b * x_out.plane;
    for (int idx = threadIdx.x; idx < TH * TW; idx += NT) {
        const int i = idx / TW, j = idx - i * TW;
        const int gr = n0 + i, gc = m0 + j;
        if (gr < R && gc < C && gr < out_h && gc < out_w)
            xp[int64_t(gr) * x_out.ld + gc] = s.in[HALO + i][HALO + j] + cols_up<UP_R>(s, up, i, j);
    }
}

__global__ __launch_bounds__(NT) void pad_fold_kernel(CView in, int R, int C, View out, int H,
                                                      int W) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const int b = blockIdx.z;
    if (c >= W) return;
    const float* ip = in.p + b * in.plane;
    const int r2 = 2 * H - 1 - r, c2 = 2 * W - 1 - c;
    float v = ip[int64_t(r) * in.ld + c];
    if (c2 < C) v += ip[int64_t(r) * in.ld + c2];
    if (r2 < R) {
        v += ip[int64_t(r2) * in.ld + c];
        if (c2 < C) v += ip[int64_t(r2) * in.ld + c2];
    }
    out.p[b * out.plane + int64_t(r) * out.ld + c] = v;
}

}  // namespace

hipError_t launch_lp_analysis(CView src, int src_h, int src_w, int pad_mode, int R, int C,
                              View c_out, View d_out, Taps5 lo, int lo_r, Taps5 up, int up_r,
                              int batch, hipStream_t st) {
    dim3 grid(((C + TW - 1) / TW) * ((R + TH - 1) / TH) * batch);
    if (lo_r == 4 && up_r == 3)
        lp_analysis_kernel<4, 3><<<grid, NT, 0, st>>>(src, src_h, src_w, pad_mode, R, C, c_out,
                                                      d_out, lo, up);
    else if (lo_r == 3 && up_r == 4)
        lp_analysis_kernel<3, 4><<<grid, NT, 0, st>>>(src, src_h, src_w, pad_mode, R, C, c_out,
                                                      d_out, lo, up);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_lp_synthesis(CView c_in, CView d_in, int R, int C, View x_out, int out_h,
                               int out_w, Taps5 lo, int lo_r, Taps5 up, int up_r, int batch,
                               hipStream_t st) {
    dim3 grid(((C + TW - 1) / TW) * ((R + TH - 1) / TH) * batch);
    if (lo_r == 4 && up_r == 3)
        lp_synthesis_kernel<4, 3><<<grid, NT, 0, st>>>(c_in, d_in, R, C, x_out, out_h, out_w, lo,
                                                       up);
    else if (lo_r == 3 && up_r == 4)
        lp_synthesis_kernel<3, 4><<<grid, NT, 0, st>>>(c_in, d_in, R, C, x_out, out_h, out_w, lo,
                                                       up);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_pad_fold(CView in, int R, int C, View out, int H, int W, int batch,
                           hipStream_t st) {
    dim3 grid((W + NT - 1) / NT, H, batch);
    pad_fold_kernel<<<grid, NT, 0, st>>>(in, R, C, out, H, W);
    return hipGetLastError();
}

}  // namespace ct

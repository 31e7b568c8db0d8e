// Fused LP level + DFB tree levels 1-2 for gfx950.
//
// Paper section 2.1: each LP level produces a half-resolution lowpass and a
// bandpass image, and the bandpass image goes through the DFB. The first two
// DFB tree levels act on the full bandpass image, so they fuse with the LP
// level that produces it: the bandpass image never leaves LDS.
//
// Analysis, per 64 x 64 tile of the level image (512 threads):
//   1. load the input tile with a 16-pixel halo (8 for the LP, 8 for the
//      eight lifting steps), periodic, with mirror or zero padding past the
//      real frame on the first level;
//   2. rows filtered by lo and decimated, then columns: the lowpass c (its
//      own 32 x 32 tile is stored);
//   3. polyphase upsampling by up and d = x - prediction on the 80 x 80 core,
//      written in place over the input;
//   4. DFB tree level 1 (cross stencil, parity n1 + n2) and level 2 (diagonal
//      stencil, parity n2), four lifting steps each, each step updating only
//      what the final 64 x 64 interior still depends on;
//   5. the four cosets of 2Z^2 leave as the tree-level-2 channels (vertical
//      ones transposed), scaled when they are already final subbands.
// Synthesis is the mirror image: the four channels are loaded with a
// 16-pixel halo, lifted back to d on the 80 x 80 core, then
// c' = c - down2(lo * d) and x = d + up * up2(c') on the 64 x 64 interior.
#include "ct_device.h"

namespace ct {
namespace {

using namespace dev;

constexpr int NT = 512;
constexpr int TO = 64;                 // output tile side
constexpr int HD = 8;                  // halo of DFB tree levels 1-2
constexpr int HL = 8;                  // halo of the LP level

// analysis tile geometry
constexpr int A_IN = TO + 2 * HD + 2 * HL;   // 96: input with both halos
constexpr int A_LD = A_IN + 1;
constexpr int A_D = TO + 2 * HD;             // 80: bandpass core fed to the DFB
constexpr int A_CN = A_D / 2 + 4;            // 44: lowpass samples per axis
constexpr int A_CLD = A_CN + 1;
constexpr int A_UHLD = A_D + 1;

struct AnaSmem {
    float in[A_IN * A_LD];
    union {
        float hf[A_IN * A_CLD];
        float uh[A_CN * A_UHLD];
    };
    float c[A_CN * A_CLD];
};

// synthesis tile geometry
constexpr int S_T = TO + 2 * HL + 2 * HD;    // 96: channel samples with both halos
constexpr int S_LD = S_T + 1;
constexpr int S_D = TO + 2 * HL;             // 80: bandpass core after lifting back
constexpr int S_CN = TO / 2 + 4;             // 36: lowpass samples per axis
constexpr int S_CLD = S_CN + 1;
constexpr int S_UHLD = TO + 1;

struct SynSmem {
    float t[S_T * S_LD];
    union {
        float hf[S_D * S_CLD];
        float uh[S_CN * S_UHLD];
    };
    float c[S_CN * S_CLD];
};

__device__ __forceinline__ void tile_of(int R, int C, int& n0, int& m0, int& b) {
    const int gx = (C + TO - 1) / TO, gy = (R + TO - 1) / TO;
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    m0 = (L % gx) * TO;
    n0 = ((L / gx) % gy) * TO;
    b = L / (gx * gy);
}

template <int LO_R, int UP_R>
__global__ __launch_bounds__(NT) void lp_dfb12_analysis_kernel(CView src, int src_h, int src_w,
                                                               int pad_mode, int R, int C,
                                                               View c_out, Quad out, Taps5 lo,
                                                               Taps5 up, Lift L) {
    __shared__ AnaSmem s;
    int n0, m0, b;
    tile_of(R, C, n0, m0, b);
    const float* sp = src.p + b * src.plane;
    constexpr int H0 = HD + HL;
    for (int idx = threadIdx.x; idx < A_IN * A_IN; idx += NT) {
        const int r = idx / A_IN, c = idx - r * A_IN;
        int gr = wrap(n0 - H0 + r, R), gc = wrap(m0 - H0 + c, C);
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
        s.in[r * A_LD + c] = v;
    }
    __syncthreads();
    rows_lo<LO_R, A_IN, A_CN, A_LD, A_CLD, NT>(s.in, s.hf, lo);
    __syncthreads();
    // lowpass sample (ss, t) is global ((n0 - 12)/2 + ss, (m0 - 12)/2 + t)
    const int Rh = R >> 1, Ch = C >> 1;
    float* cp = c_out.p + b * c_out.plane;
    for (int idx = threadIdx.x; idx < A_CN * A_CN; idx += NT) {
        const int ss = idx / A_CN, t = idx - ss * A_CN;
        const float v = cols_lo<LO_R, A_CLD>(s.hf, lo, ss, t);
        s.c[ss * A_CLD + t] = v;
        constexpr int OFF = (HD + 4) / 2;   // 6: first owned lowpass sample
        if (ss >= OFF && ss < OFF + TO / 2 && t >= OFF && t < OFF + TO / 2) {
            const int gr = (n0 >> 1) + ss - OFF, gc = (m0 >> 1) + t - OFF;
            if (gr < Rh && gc < Ch) cp[int64_t(gr) * c_out.ld + gc] = v;
        }
    }
    __syncthreads();
    rows_up<UP_R, A_CN, A_D, A_CLD, A_UHLD, NT>(s.c, s.uh, up);
    __syncthreads();
    float* T = s.in + HL * A_LD + HL;          // the 80 x 80 bandpass core
    for (int idx = threadIdx.x; idx < A_D * A_D; idx += NT) {
        const int i = idx / A_D, j = idx - i * A_D;
        T[i * A_LD + j] -= cols_up<UP_R, A_UHLD>(s.uh, up, i, j);
    }
    __syncthreads();
    int m = 1;
    for (int st = 0; st < 4; ++st, ++m) {
        step_cross<A_D, A_LD, NT>(T, (L.first_odd + st) & 1, 0.5f * L.c[st], m);
        __syncthreads();
    }
    for (int st = 0; st < 4; ++st, ++m) {
        step_diag<A_D, A_LD, NT>(T, (L.first_odd + st) & 1, 0.5f * L.c[st], m);
        __syncthreads();
    }
    constexpr int HQ = TO / 2;
    // horizontal channels, row major (R/2) x (C/2): quad 0 = coset (0,1), 1 = (1,0)
    for (int idx = threadIdx.x; idx < 2 * HQ * HQ; idx += NT) {
        const int q = idx / (HQ * HQ);
        const int rem = idx - q * HQ * HQ;
        const int i = rem / HQ, k = rem - i * HQ;
        const int pr = q == 0 ? 0 : 1, pc = q == 0 ? 1 : 0;
        const int gi = (n0 >> 1) + i, gk = (m0 >> 1) + k;
        if (gi < Rh && gk < Ch)
            out.p[q][b * out.plane + int64_t(gi) * Ch + gk] =
                out.scale[q] * T[(HD + 2 * i + pr) * A_LD + HD + 2 * k + pc];
    }
    // vertical channels, transposed (C/2) x (R/2): quad 2 = coset (0,0), 3 = (1,1)
    for (int idx = threadIdx.x; idx < 2 * HQ * HQ; idx += NT) {
        const int q = 2 + idx / (HQ * HQ);
        const int rem = idx - (q - 2) * HQ * HQ;
        const int k = rem / HQ, i = rem - k * HQ;
        const int p = q == 2 ? 0 : 1;
        const int gi = (n0 >> 1) + i, gk = (m0 >> 1) + k;
        if (gi < Rh && gk < Ch)
            out.p[q][b * out.plane + int64_t(gk) * Rh + gi] =
                out.scale[q] * T[(HD + 2 * i + p) * A_LD + HD + 2 * k + p];
    }
}

template <int LO_R, int UP_R>
__global__ __launch_bounds__(NT) void dfb12_lp_synthesis_kernel(Quad in, CView c_in, int R, int C,
                                                                View x_out, int out_h, int out_w,
                                                                Taps5 lo, Taps5 up, Lift L) {
    __shared__ SynSmem s;
    int n0, m0, b;
    tile_of(R, C, n0, m0, b);
    const int Rh = R >> 1, Ch = C >> 1;
    constexpr int HN = S_T / 2;                // 48 compact samples per axis
    constexpr int H0 = (HD + HL) / 2;          // 8: compact halo
    // horizontal channels (row major): lanes along compact columns
    for (int idx = threadIdx.x; idx < 2 * HN * HN; idx += NT) {
        const int q = idx / (HN * HN);
        const int rem = idx - q * HN * HN;
        const int i = rem / HN, k = rem - i * HN;
        const int pr = q == 0 ? 0 : 1, pc = q == 0 ? 1 : 0;
        const int gi = wrap((n0 >> 1) - H0 + i, Rh), gk = wrap((m0 >> 1) - H0 + k, Ch);
        s.t[(2 * i + pr) * S_LD + 2 * k + pc] = in.scale[q] * in.p[q][b * in.plane + int64_t(gi) * Ch + gk];
    }
    // vertical channels (transposed): lanes along compact rows
    for (int idx = threadIdx.x; idx < 2 * HN * HN; idx += NT) {
        const int q = 2 + idx / (HN * HN);
        const int rem = idx - (q - 2) * HN * HN;
        const int k = rem / HN, i = rem - k * HN;
        const int p = q == 2 ? 0 : 1;
        const int gi = wrap((n0 >> 1) - H0 + i, Rh), gk = wrap((m0 >> 1) - H0 + k, Ch);
        s.t[(2 * i + p) * S_LD + 2 * k + p] = in.scale[q] * in.p[q][b * in.plane + int64_t(gk) * Rh + gi];
    }
    // lowpass tile: rows/cols (n0/2 - 2 .. n0/2 + 34)
    const float* cp = c_in.p + b * c_in.plane;
    for (int idx = threadIdx.x; idx < S_CN * S_CN; idx += NT) {
        const int ss = idx / S_CN, t = idx - ss * S_CN;
        const int gr = wrap((n0 >> 1) - 2 + ss, Rh), gc = wrap((m0 >> 1) - 2 + t, Ch);
        s.c[ss * S_CLD + t] = cp[int64_t(gr) * c_in.ld + gc];
    }
    __syncthreads();
    int m = 1;
    for (int st = 0; st < 4; ++st, ++m) {
        step_diag<S_T, S_LD, NT>(s.t, (L.first_odd + st) & 1, 0.5f * L.c[st], m);
        __syncthreads();
    }
    for (int st = 0; st < 4; ++st, ++m) {
        step_cross<S_T, S_LD, NT>(s.t, (L.first_odd + st) & 1, 0.5f * L.c[st], m);
        __syncthreads();
    }
    const float* D = s.t + HD * S_LD + HD;     // the 80 x 80 bandpass core
    rows_lo<LO_R, S_D, S_CN, S_LD, S_CLD, NT>(D, s.hf, lo);
    __syncthreads();
    for (int idx = threadIdx.x; idx < S_CN * S_CN; idx += NT) {
        const int ss = idx / S_CN, t = idx - ss * S_CN;
        s.c[ss * S_CLD + t] -= cols_lo<LO_R, S_CLD>(s.hf, lo, ss, t);
    }
    __syncthreads();
    rows_up<UP_R, S_CN, TO, S_CLD, S_UHLD, NT>(s.c, s.uh, up);
    __syncthreads();
    float* xp = x_out.p + b * x_out.plane;
    for (int idx = threadIdx.x; idx < TO * TO; idx += NT) {
        const int i = idx / TO, j = idx - i * TO;
        const int gr = n0 + i, gc = m0 + j;
        if (gr < R && gc < C && gr < out_h && gc < out_w)
            xp[int64_t(gr) * x_out.ld + gc] = D[(HL + i) * S_LD + HL + j] + cols_up<UP_R, S_UHLD>(s.uh, up, i, j);
    }
}

}  // namespace

hipError_t launch_lp_dfb12_analysis(CView src, int src_h, int src_w, int pad_mode, int R, int C,
                                    View c_out, Quad out, Taps5 lo, int lo_r, Taps5 up, int up_r,
                                    Lift lift, int batch, hipStream_t st) {
    dim3 grid(((C + TO - 1) / TO) * ((R + TO - 1) / TO) * batch);
    if (lo_r == 4 && up_r == 3)
        lp_dfb12_analysis_kernel<4, 3><<<grid, NT, 0, st>>>(src, src_h, src_w, pad_mode, R, C,
                                                            c_out, out, lo, up, lift);
    else if (lo_r == 3 && up_r == 4)
        lp_dfb12_analysis_kernel<3, 4><<<grid, NT, 0, st>>>(src, src_h, src_w, pad_mode, R, C,
                                                            c_out, out, lo, up, lift);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_dfb12_lp_synthesis(Quad in, CView c_in, int R, int C, View x_out, int out_h,
                                     int out_w, Taps5 lo, int lo_r, Taps5 up, int up_r, Lift lift,
                                     int batch, hipStream_t st) {
    dim3 grid(((C + TO - 1) / TO) * ((R + TO - 1) / TO) * batch);
    if (lo_r == 4 && up_r == 3)
        dfb12_lp_synthesis_kernel<4, 3><<<grid, NT, 0, st>>>(in, c_in, R, C, x_out, out_h, out_w,
                                                             lo, up, lift);
    else if (lo_r == 3 && up_r == 4)
        dfb12_lp_synthesis_kernel<3, 4><<<grid, NT, 0, st>>>(in, c_in, R, C, x_out, out_h, out_w,
                                                             lo, up, lift);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace ct

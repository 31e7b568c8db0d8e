// Register-streaming form of one LP level fused with DFB tree levels 1 and 2
// (analysis), for gfx950.
//
// Paper section 2.1 (Laplacian pyramid, then the DFB on the bandpass image,
// 9-7 filters), section 3.3 (the lowpass at half resolution per level).
//
// A wavefront owns a strip of 128 image columns (lane l holds columns
// 2l and 2l + 1, i.e. lowpass column l) and streams down a block of rows.
// Per pair of image rows (a superstep):
//   hf  = horizontal lowpass of each new row            (lanes via DPP)
//   c   = vertical lowpass of hf, one lowpass row         (register ring)
//   uh  = horizontal upsampling of that lowpass row       (DPP)
//   d   = x - vertical upsampling of uh, two bandpass rows
//   DFB tree level 1 (4 lifting steps), level 2 (4 steps), each one row
//       further behind than the previous, on the d rows
// and the two rows leaving the last step are the four quarter channels of
// tree level 2. Horizontal-cone channels are stored row by row; the
// vertical-cone ones are stored transposed, so they are gathered in a
// wave-private LDS block of 16 compact rows and written out column-wise.
//
// Lags (rows behind the newest loaded row 2n + 1, relative to the first
// streamed row): c row n - 2, d rows 2n - 8 and 2n - 7, final rows 2n - 16
// and 2n - 15. An output row depends on input rows from 17 above to 16
// below it; blocks load 18 rows above and 16 below, and 16 columns on each
// side of the 96 columns they store.
#pragma once

#include "ct_color_stages.h"
#include "ct_quant_stages.h"
#include "ct_stream.h"

namespace ct {
namespace stream {

// Horizontal lowpass at lowpass column l (image column 2l):
// sum_k lo[k] x[2l +- k].
template <int LO_R>
__device__ __forceinline__ float row_lowpass(const Taps5& lo, float x0, float x1) {
    const float p1 = from_prev(x1);                         // x[2l - 1]
    const float n0 = from_next(x0), p0 = from_prev(x0);     // x[2l + 2], x[2l - 2]
    float acc = lo.t[0] * x0;
    acc = fmaf(lo.t[1], p1 + x1, acc);
    acc = fmaf(lo.t[2], p0 + n0, acc);
    if (LO_R >= 3) acc = fmaf(lo.t[3], from_prev(p1) + from_next(x1), acc);   // x[2l - 3], x[2l + 3]
    if (LO_R >= 4) acc = fmaf(lo.t[4], from_prev(p0) + from_next(n0), acc);   // x[2l - 4], x[2l + 4]
    return acc;
}

// Vertical lowpass from 2 LO_R + 1 rows h[0..2 LO_R] centred on h[LO_R].
template <int LO_R>
__device__ __forceinline__ float col_lowpass(const Taps5& lo, const float* h) {
    float acc = lo.t[0] * h[LO_R];
#pragma unroll
    for (int k = 1; k <= LO_R; ++k) acc = fmaf(lo.t[k], h[LO_R - k] + h[LO_R + k], acc);
    return acc;
}

// Horizontal upsampling of a lowpass row (value c at lowpass column l, i.e.
// image column 2l): outputs at image columns 2l (.x) and 2l + 1 (.y).
template <int UP_R>
__device__ __forceinline__ Pair row_upsample(const Taps5& up, float c) {
    const float cn = from_next(c), cp = from_prev(c);   // c[l + 1], c[l - 1]
    Pair r;
    float e = up.t[0] * c;
    e = fmaf(up.t[2], cp + cn, e);
    float o = up.t[1] * (c + cn);
    if (UP_R >= 3) o = fmaf(up.t[3], cp + from_next(cn), o);   // c[l - 1], c[l + 2]
    if (UP_R >= 4) e = fmaf(up.t[4], from_prev(cp) + from_next(cn), e);
    r.x = e;
    r.y = o;
    return r;
}

template <int LO_R, int UP_R, int NT>
struct StreamLevelAna {
    static constexpr int WAVES = NT / 64;
    static constexpr int HC = 16;            // halo image columns on each side
    static constexpr int VW = level_cols();  // stored image columns per strip (128 - 2 HC)
    static constexpr int TOP = 18;           // rows loaded above a block
    static constexpr int LAG = 16;           // rows from the newest loaded row to the output
    static constexpr int PF = 2;             // supersteps of prefetched input rows
    static constexpr int U = 5 + PF;         // supersteps per ring cycle
    static constexpr int RR = 2 * U;         // ring rows: x (12 in use plus the prefetched), hf and d
    static constexpr int RC = U;             // ring rows: uh (lowpass rows)
    static constexpr int VB = 16;            // compact rows per transposed flush
    static constexpr int VLD = VB + 1;
    static constexpr int WAVE_SMEM = 2 * 64 * VLD;
    static constexpr int SMEM = WAVES * WAVE_SMEM;   // floats

    const stage::LevelAnaArgs& A;
    __device__ StreamLevelAna(const stage::LevelAnaArgs& a) : A(a) {}

    static_assert(VW == 128 - 2 * HC, "strip geometry");
    __device__ int strips() const { return (A.C + VW - 1) / VW; }
    __device__ int blocks() const { return (A.R + A.bh - 1) / A.bh; }
    __device__ int items() const { return level_items(A.R, A.C, A.batch, A.bh); }
    __device__ int tiles() const { return (items() + WAVES - 1) / WAVES; }

    static constexpr int rslot(int rel) { return ((rel % RR) + RR) % RR; }
    static constexpr int cslot(int rel) { return ((rel % RC) + RC) % RC; }

    // QOUT must match A.q.idx != nullptr and RGB A.rgb != nullptr (the
    // launcher picks the kernel).
    template <bool QOUT, bool RGB = false>
    __device__ __forceinline__ void run_tile(int tile, float* smem) const {
        const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
        const int item = tile * WAVES + wave;
        if (item < items()) {
            float* T = smem + wave * WAVE_SMEM;
            if (A.L.first_odd) run<1, QOUT, RGB>(item, T);
            else run<0, QOUT, RGB>(item, T);
        }
    }

    // QOUT: the four channels are final subbands quantised on store. RGB:
    // the source is the RGB frames, each plane one channel (forward
    // transform, mirror padding).
    template <int FO, bool QOUT, bool RGB>
    __device__ __forceinline__ void run(int item, float* T) const {
        const int ns = strips(), nb = blocks();
        const int b = item / (ns * nb);
        const int rem = item - b * ns * nb;
        const int blk = rem / ns, strip = rem - blk * ns;
        const int R = A.R, C = A.C, Rh = R >> 1, Ch = C >> 1;
        const int kb = strip * VW, rb = blk * A.bh;
        const int re = min(rb + A.bh, R);
        const int lane = threadIdx.x & 63;
        const int cb0 = kb - HC;                    // image column of lane 0's x0 (even)
        const int kc = (cb0 >> 1) + lane;           // this lane's compact column (unwrapped)
        const bool own = lane >= HC / 2 && lane < 64 - HC / 2 && kc < Ch;
        const int S = rb - TOP;                     // first streamed row (even)
        const int NS = (re - rb) / 2 + (TOP - 1);   // supersteps until the last output row

        // source columns of the lane's two image columns (periodic, then
        // padded past the real frame); zero padding clears the loaded bits
        // with a mask, so every load is unconditional
        const float* sp = RGB ? nullptr : A.src.p + b * A.src.plane;
        uint32_t sc[2];                             // byte offsets within a source row
        uint32_t mc[2];
        // RGB source: frame b / 3, channel b % 3 as ((wr r + wg g) + wb b) + w0,
        // the operations of equations (1)-(3) (exact in float32)
        const uint8_t* fp = RGB ? A.rgb + int64_t(b / 3) * (3 * int64_t(A.src_h) * A.src_w) : nullptr;
        const int ch = b - 3 * (b / 3);
        const float wr = ch == 0 ? 0.25f : ch == 1 ? 0.5f : -0.25f;
        const float wg = ch == 0 ? 0.5f : ch == 1 ? 0.f : 0.5f;
        const float wb = ch == 0 ? 0.25f : ch == 1 ? -0.5f : -0.25f;
        const float w0 = ch == 0 ? 0.f : color::kChromaOffset;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            int g = pmod(cb0 + 2 * lane + e, C);
            mc[e] = ~0u;
            if (A.pad_mode == kPadReflect && g >= A.src_w) g = 2 * A.src_w - 1 - g;
            if (A.pad_mode == kPadZero && g >= A.src_w) {
                mc[e] = 0u;
                g = 0;
            }
            sc[e] = (RGB ? 3u : 4u) * uint32_t(g);
        }
        int xrow = pmod(S, R);                      // next row to load, modulo R
        auto load_row = [&](Pair& X) {
            int g = xrow;
            uint32_t mr = ~0u;
            if (A.pad_mode == kPadReflect && g >= A.src_h) g = 2 * A.src_h - 1 - g;
            if (A.pad_mode == kPadZero && g >= A.src_h) {
                mr = 0u;
                g = 0;
            }
            if constexpr (RGB) {
                // reflect padding only: the masks are all ones
                const uint8_t* rp = fp + int64_t(g) * (3 * A.src_w);
                float v[2];
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const float r = float(ld_at(rp, sc[e])), gg = float(ld_at(rp, sc[e] + 1u));
                    const float bb = float(ld_at(rp, sc[e] + 2u));
                    v[e] = __fadd_rn(__fadd_rn(__fadd_rn(__fmul_rn(wr, r), __fmul_rn(wg, gg)), __fmul_rn(wb, bb)), w0);
                }
                X.x = v[0];
                X.y = v[1];
            } else {
                const uint32_t* rp = reinterpret_cast<const uint32_t*>(sp + int64_t(g) * A.src.ld);
                X.x = __uint_as_float(ld_at(rp, sc[0]) & (mr & mc[0]));
                X.y = __uint_as_float(ld_at(rp, sc[1]) & (mr & mc[1]));
            }
            xrow = xrow + 1 == R ? 0 : xrow + 1;
        };

        float* cp = A.c_out.p + b * A.c_out.plane;
        // the four channels as floats (out.p[0] null: not written) and, for a
        // level with four directions under the encoder, as indices
        const bool fout = A.out.p[0] != nullptr;
        float* q0 = fout ? A.out.p[0] + b * A.out.plane : nullptr;
        float* q1 = fout ? A.out.p[1] + b * A.out.plane : nullptr;
        float* q2 = fout ? A.out.p[2] + b * A.out.plane : nullptr;
        float* q3 = fout ? A.out.p[3] + b * A.out.plane : nullptr;
        const float s0 = A.out.scale[0], s1 = A.out.scale[1];
        const float s2 = A.out.scale[2], s3 = A.out.scale[3];
        constexpr bool qout = QOUT;
        const int64_t q4 = int64_t(Rh) * Ch;
        int16_t* x0 = qout ? A.q.idx + b * A.q.plane : nullptr;
        const float* qst = qout ? A.q.steps + int64_t(b) * A.q.steps_stride + A.q.sub0 : nullptr;
        const float d0 = qout ? qst[0] : 1.f, d1 = qout ? qst[1] : 1.f;
        const float d2 = qout ? qst[2] : 1.f, d3 = qout ? qst[3] : 1.f;
        const bool qfast = qout && __builtin_amdgcn_readfirstlane(int(qstage::fast_step(d0) && qstage::fast_step(d1) &&
                                                                       qstage::fast_step(d2) && qstage::fast_step(d3))) != 0;
        const float r0 = qfast ? __fdiv_rn(1.f, d0) : 1.f, r1 = qfast ? __fdiv_rn(1.f, d1) : 1.f;
        const float r2 = qfast ? __fdiv_rn(1.f, d2) : 1.f, r3 = qfast ? __fdiv_rn(1.f, d3) : 1.f;
        const uint32_t kc4 = 4u * uint32_t(kc), kc2 = 2u * uint32_t(kc);   // owning lanes: kc >= 0

        // transposed flush of `cnt` compact rows starting at compact row i0:
        // four compact columns per instruction, VB rows each
        auto flush = [&](int i0, int cnt) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const int li = lane & (VB - 1), lk = lane >> 4;
            // element offset of the lane's first stored (column, row) within
            // a channel, column (cb0 >> 1) + HC / 2 + lk >= 0 (a channel holds
            // fewer than 2^28 elements, so byte offsets fit 32 bits); group kk
            // adds (kk - HC / 2) Rh
            const uint32_t lo = uint32_t((cb0 >> 1) + HC / 2 + lk) * uint32_t(Rh) + uint32_t(li);
#pragma unroll
            for (int kk = HC / 2; kk < 64 - HC / 2; kk += 4) {
                const int l = kk + lk;
                const int k = (cb0 >> 1) + l;
                if (li < cnt && k < Ch) {
                    const int64_t ob = int64_t(kk - HC / 2) * Rh + i0;   // wave-uniform part
                    const float a = T[l * VLD + li], e = T[(64 + l) * VLD + li];
                    if (fout) {
                        st_at(q2 + ob, 4u * lo, a);
                        st_at(q3 + ob, 4u * lo, e);
                    }
                    if (qout) {
                        st_at(x0 + 2 * q4 + ob, 2u * lo, qstage::index_of(a, d2, r2, qfast));
                        st_at(x0 + 3 * q4 + ob, 2u * lo, qstage::index_of(e, d3, r3, qfast));
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };

        Pair xr[RR], dr[RR];
        float hf[RR];
        Pair uh[RC];
#pragma unroll
        for (int r = 0; r < RR; ++r) {
            xr[r] = Pair{0.f, 0.f};
            dr[r] = Pair{0.f, 0.f};
            hf[r] = 0.f;
        }
#pragma unroll
        for (int r = 0; r < RC; ++r) uh[r] = Pair{0.f, 0.f};

#pragma unroll
        for (int r = 0; r < 2 * PF; ++r) load_row(xr[r]);
        for (int n0 = 0; n0 < NS; n0 += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int n = n0 + u;
                // prefetch the pair of rows PF supersteps ahead
                load_row(xr[rslot(2 * u + 2 * PF)]);
                load_row(xr[rslot(2 * u + 2 * PF + 1)]);
                // horizontal lowpass of rows 2n, 2n + 1
                hf[rslot(2 * u)] = row_lowpass<LO_R>(A.lo, xr[rslot(2 * u)].x, xr[rslot(2 * u)].y);
                hf[rslot(2 * u + 1)] =
                    row_lowpass<LO_R>(A.lo, xr[rslot(2 * u + 1)].x, xr[rslot(2 * u + 1)].y);
                // lowpass row n - 2 from hf rows 2n - 8 .. 2n
                float h[2 * LO_R + 1];
#pragma unroll
                for (int k = 0; k <= 2 * LO_R; ++k) h[k] = hf[rslot(2 * u - 4 - LO_R + k)];
                const float cv = col_lowpass<LO_R>(A.lo, h);
                {
                    const int s = (S >> 1) + n - 2;
                    if (own && s >= (rb >> 1) && s < (re >> 1)) st_at(cp + int64_t(s) * A.c_out.ld, kc4, cv);
                }
                uh[cslot(u - 2)] = row_upsample<UP_R>(A.up, cv);
                // bandpass rows 2m, 2m + 1 with m = n - 4
                {
                    const Pair um2 = uh[cslot(u - 6)], um1 = uh[cslot(u - 5)], u0 = uh[cslot(u - 4)];
                    const Pair up1 = uh[cslot(u - 3)], up2 = uh[cslot(u - 2)];
                    const Pair xe = xr[rslot(2 * u - 8)], xo = xr[rslot(2 * u - 7)];
                    Pair de, dod;
                    float ex = A.up.t[0] * u0.x, ey = A.up.t[0] * u0.y;
                    ex = fmaf(A.up.t[2], um1.x + up1.x, ex);
                    ey = fmaf(A.up.t[2], um1.y + up1.y, ey);
                    if (UP_R >= 4) {
                        ex = fmaf(A.up.t[4], um2.x + up2.x, ex);
                        ey = fmaf(A.up.t[4], um2.y + up2.y, ey);
                    }
                    float ox = A.up.t[1] * (u0.x + up1.x), oy = A.up.t[1] * (u0.y + up1.y);
                    ox = fmaf(A.up.t[3], um1.x + up2.x, ox);
                    oy = fmaf(A.up.t[3], um1.y + up2.y, oy);
                    de.x = xe.x - ex;
                    de.y = xe.y - ey;
                    dod.x = xo.x - ox;
                    dod.y = xo.y - oy;
                    dr[rslot(2 * u - 8)] = de;
                    dr[rslot(2 * u - 7)] = dod;
                }
                // DFB tree level 1 then level 2, step q on rows 2n - 9 - q, 2n - 8 - q
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int st = q & 3;
                    const float cf = 0.5f * A.L.c[st];
                    const int par = (FO + st) & 1;
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int rel = 2 * u - 9 - q + j;          // row parity = (1 + q + j) & 1
                        const int rpar = (((-9 - q + j) % 2) + 2) % 2;
                        Pair& X = dr[rslot(rel)];
                        const Pair& Up = dr[rslot(rel - 1)];
                        const Pair& Dn = dr[rslot(rel + 1)];
                        if (q < 4) {
                            // points with (row + column) & 1 == par
                            if (rpar == par) X.x = fmaf(cf, (X.y + from_prev(X.y)) - (Dn.x + Up.x), X.x);
                            else X.y = fmaf(cf, (from_next(X.x) + X.x) - (Dn.y + Up.y), X.y);
                        } else {
                            // points with column & 1 == par
                            if (par == 0)
                                X.x = fmaf(cf, (Up.y + from_prev(Dn.y)) - (Dn.y + from_prev(Up.y)), X.x);
                            else
                                X.y = fmaf(cf, (from_next(Up.x) + Dn.x) - (from_next(Dn.x) + Up.x), X.y);
                        }
                    }
                }
                // rows 2n - 16 (even) and 2n - 15 (odd) are final: compact row i
                {
                    const int i = (S >> 1) + n - (LAG >> 1);
                    if (i >= (rb >> 1) && i < (re >> 1)) {
                        const Pair E = dr[rslot(2 * u - 16)], O = dr[rslot(2 * u - 15)];
                        if (own) {
                            const float a = s0 * E.y, e = s1 * O.x;
                            const int64_t o = int64_t(i) * Ch;
                            if (fout) {
                                st_at(q0 + o, kc4, a);
                                st_at(q1 + o, kc4, e);
                            }
                            if (qout) {
                                st_at(x0 + o, kc2, qstage::index_of(a, d0, r0, qfast));
                                st_at(x0 + q4 + o, kc2, qstage::index_of(e, d1, r1, qfast));
                            }
                        }
                        const int slot = (i - (rb >> 1)) & (VB - 1);
                        T[lane * VLD + slot] = s2 * E.x;
                        T[(64 + lane) * VLD + slot] = s3 * O.y;
                        if (slot == VB - 1 || i == (re >> 1) - 1) flush(i - slot, slot + 1);
                    }
                }
            }
        }
    }
};

}  // namespace stream
}  // namespace ct

namespace ct {
namespace stream {

// DFB tree levels 2 and 1 back to the bandpass image, then the dual LP
// synthesis, in the same streaming layout (paper section 2.1: perfect
// reconstruction of the LP and DFB). Per compact row n of the four quarter
// channels (image rows 2n, 2n + 1):
//   place the channels on the checkerboard, tree level 2 (4 steps) and
//   level 1 (4 steps) one row further behind each -> bandpass rows 2n - 8,
//   2n - 7; hf = horizontal lowpass of those rows; c' = c - vertical
//   lowpass of hf (lowpass row n - 6); uh = horizontal upsampling of c';
//   x = d + vertical upsampling of uh: image rows 2n - 16, 2n - 15.
// The vertical-cone channels are stored transposed; blocks of VB = 16
// compact rows of them are staged through wave-private LDS. A block's loads
// are issued into registers when the previous block starts and written to
// LDS when their own block starts; aligned blocks that do not wrap are read
// as 16-byte pieces (four lanes per 64-byte column run).
template <int LO_R, int UP_R, int NT>
struct StreamLevelSyn {
    static constexpr int WAVES = NT / 64;
    static constexpr int HC = 16;
    static constexpr int VW = level_cols();
    static constexpr int TOP = 16;           // an output row depends on input rows 15 above it
    static constexpr int LAG = 16;
    static constexpr int U = 10;             // supersteps per ring cycle
    static constexpr int PFH = 5;            // supersteps of prefetched H and lowpass rows
    static constexpr int RR = 20;            // ring rows: channels / bandpass
    static constexpr int RH = 10;            // ring rows: hf
    static constexpr int RC = 5;             // ring rows: uh (lowpass rows)
    static constexpr int VB = 16;            // compact rows per staged block
    static constexpr int VLD = VB + 1;
    static constexpr int BUF = 2 * 64 * VLD; // one staged block, both channels
    static constexpr int WAVE_SMEM = BUF;
    static constexpr int SMEM = WAVES * WAVE_SMEM;
    static constexpr int NSTAGE = 2 * 64 * VB / 64;   // staged values per lane per block

    const stage::LevelSynArgs& A;
    __device__ StreamLevelSyn(const stage::LevelSynArgs& a) : A(a) {}

    static_assert(VW == 128 - 2 * HC, "strip geometry");
    __device__ int strips() const { return (A.C + VW - 1) / VW; }
    __device__ int blocks() const { return (A.R + A.bh - 1) / A.bh; }
    __device__ int items() const { return level_items(A.R, A.C, A.batch, A.bh); }
    __device__ int tiles() const { return (items() + WAVES - 1) / WAVES; }

    static constexpr int rslot(int rel) { return ((rel % RR) + RR) % RR; }
    static constexpr int hslot(int rel) { return ((rel % RH) + RH) % RH; }
    static constexpr int cslot(int rel) { return ((rel % RC) + RC) % RC; }

    // QIN must match (A.q.idx or A.lq.idx) != nullptr (the launcher picks the kernel);
    // LOWONLY: only the lowpass is indices (A.q.idx null), fixed at compile time.
    template <bool QIN, bool LOWONLY = false>
    __device__ __forceinline__ void run_tile(int tile, float* smem) const {
        const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
        const int item = tile * WAVES + wave;
        if (item < items()) {
            float* T = smem + wave * WAVE_SMEM;
            if (A.L.first_odd) run<1, QIN, LOWONLY>(item, T);
            else run<0, QIN, LOWONLY>(item, T);
        }
    }

    // QIN: the four channels and / or the lowpass are indices dequantised on load
    template <int FO, bool QIN, bool LOWONLY>
    __device__ __forceinline__ void run(int item, float* T) const {
        const int ns = strips(), nb = blocks();
        const int b = item / (ns * nb);
        const int rem = item - b * ns * nb;
        const int blk = rem / ns, strip = rem - blk * ns;
        const int R = A.R, C = A.C, Rh = R >> 1, Ch = C >> 1;
        const int kb = strip * VW, rb = blk * A.bh;
        const int re = min(rb + A.bh, R);
        const int lane = threadIdx.x & 63;
        const int cb0 = kb - HC;
        const int kcw = pmod((cb0 >> 1) + lane, Ch);     // compact column, wrapped
        const int S2 = (rb - TOP) >> 1;                  // first streamed compact row (0 mod 4)
        const int NS = (re - rb) / 2 + (TOP + LAG) / 2;  // the first output pair leaves at n = 16
        const int ow = min(A.out_w, C), oh = min(A.out_h, R);
        const bool own = lane >= HC / 2 && lane < 64 - HC / 2;
        const int j0 = cb0 + 2 * lane;                   // image columns j0, j0 + 1
        const bool st0 = own && j0 < ow, st1 = own && j0 + 1 < ow;
        const uint32_t j4 = 4u * uint32_t(j0);           // used by storing lanes only (j0 >= 0)
        const bool pair_st = (ow & 1) == 0;

        // the four channels as floats, or (decoder, levels with four
        // directions) as indices dequantised on load
        const bool qin = QIN && !LOWONLY && A.q.idx != nullptr;
        const float* h0 = qin ? nullptr : A.in.p[0] + b * A.in.plane;   // H a=-1: even rows, odd columns
        const float* h1 = qin ? nullptr : A.in.p[1] + b * A.in.plane;   // H a=0:  odd rows, even columns
        const float* v2 = qin ? nullptr : A.in.p[2] + b * A.in.plane;   // V a=0:  even rows, even columns
        const float* v3 = qin ? nullptr : A.in.p[3] + b * A.in.plane;   // V a=-1: odd rows, odd columns
        const float s0 = A.in.scale[0], s1 = A.in.scale[1];
        const float s2 = A.in.scale[2], s3 = A.in.scale[3];
        const int64_t q4 = int64_t(Rh) * Ch;
        const int16_t* x0 = qin ? A.q.idx + b * A.q.plane : nullptr;
        const float* qst = qin ? A.q.steps + int64_t(b) * A.q.steps_stride + A.q.sub0 : nullptr;
        const float d0 = qin ? qst[0] : 1.f, d1 = qin ? qst[1] : 1.f;
        const float d2 = qin ? qst[2] : 1.f, d3 = qin ? qst[3] : 1.f;
        // the lowpass c_in as floats, or (decoder, coarsest level) as indices
        const bool lin = QIN && (LOWONLY || A.lq.idx != nullptr);
        const float* cin = lin ? nullptr : A.c_in.p + b * A.c_in.plane;
        const int16_t* lx = lin ? A.lq.idx + b * A.lq.plane : nullptr;
        float l_mn = 0.f, l_step = 1.f, l_r = 0.f;
        if (lin) {
            l_mn = A.side[2 * b];
            const float l_mx = A.side[2 * b + 1];
            l_step = A.lq.steps[int64_t(b) * A.lq.steps_stride];
            l_r = __fdiv_rn(__fsub_rn(l_mx, l_mn), 255.f);
        }
        float* xo = A.x_out.p + b * A.x_out.plane;

        // Staging of the transposed channels, compact rows [i0, i0 + 16) of the
        // strip's 64 compact columns: lane (cg, rc) holds rows i0 + 4 rc .. + 3
        // of columns 16 c + cg, c = 0..3. Blocks aligned to 4 rows and inside
        // the array are read as one 16-byte load per column; wrapping or
        // unaligned blocks element by element.
        const bool vec_ok = !qin && (Rh & 3) == 0 &&
                            ((reinterpret_cast<uintptr_t>(v2) | reinterpret_cast<uintptr_t>(v3)) & 15) == 0;
        const int cg = lane >> 2, rc = lane & 3;
        // element offsets of the lane's four columns within a channel (a
        // channel holds fewer than 2^28 elements, so byte offsets fit 32 bits)
        uint32_t kcol[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) kcol[c] = uint32_t(pmod((cb0 >> 1) + 16 * c + cg, Ch)) * uint32_t(Rh);
        float stg[NSTAGE];
        const int16_t* x2 = qin ? x0 + 2 * q4 : nullptr;
        const int16_t* x3 = qin ? x0 + 3 * q4 : nullptr;
        auto stage_load = [&](int i0) {
            if (vec_ok && i0 >= 0 && i0 + VB <= Rh) {
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const uint32_t o = 4u * (kcol[c] + 4 * rc);
                    const float4 a = ld_at(reinterpret_cast<const float4*>(v2 + i0), o);
                    const float4 e = ld_at(reinterpret_cast<const float4*>(v3 + i0), o);
                    stg[4 * c + 0] = a.x;
                    stg[4 * c + 1] = a.y;
                    stg[4 * c + 2] = a.z;
                    stg[4 * c + 3] = a.w;
                    stg[16 + 4 * c + 0] = e.x;
                    stg[16 + 4 * c + 1] = e.y;
                    stg[16 + 4 * c + 2] = e.z;
                    stg[16 + 4 * c + 3] = e.w;
                }
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t i = uint32_t(pmod(i0 + 4 * rc + e, Rh));
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        if (qin) {
                            stg[4 * c + e] = __fmul_rn(float(ld_at(x2, 2u * (kcol[c] + i))), d2);
                            stg[16 + 4 * c + e] = __fmul_rn(float(ld_at(x3, 2u * (kcol[c] + i))), d3);
                        } else {
                            stg[4 * c + e] = ld_at(v2, 4u * (kcol[c] + i));
                            stg[16 + 4 * c + e] = ld_at(v3, 4u * (kcol[c] + i));
                        }
                    }
                }
            }
        };
        auto stage_store = [&]() {
            float* Tl = T + cg * VLD + 4 * rc;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    Tl[16 * c * VLD + e] = stg[4 * c + e];
                    Tl[(64 + 16 * c) * VLD + e] = stg[16 + 4 * c + e];
                }
            }
        };
        auto lds_sync = [&]() {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        };

        int hrow = pmod(S2, Rh);            // next compact row of the H channels
        int crow = pmod(S2 - 6, Rh);        // next lowpass row
        // H values and lowpass values of the compact rows two supersteps
        // ahead, as loaded (indices keep their integer bits and are
        // dequantised where they are used, so nothing waits on a load early)
        Pair hq[PFH];
        float cq[PFH];
        const uint32_t kcw4 = 4u * uint32_t(kcw), kcw2 = 2u * uint32_t(kcw);
        auto load_h = [&](Pair& hn) {
            const int64_t o = int64_t(hrow) * Ch;
            if (qin) {
                hn.x = __builtin_bit_cast(float, int(ld_at(x0 + q4 + o, kcw2)));   // odd row, even column
                hn.y = __builtin_bit_cast(float, int(ld_at(x0 + o, kcw2)));        // even row, odd column
            } else {
                hn.x = ld_at(h1 + o, kcw4);
                hn.y = ld_at(h0 + o, kcw4);
            }
            hrow = hrow + 1 == Rh ? 0 : hrow + 1;
        };
        auto load_c = [&](float& cn) {
            if (lin) cn = __builtin_bit_cast(float, int(ld_at(lx + int64_t(crow) * A.c_in.ld, kcw2)));
            else cn = ld_at(cin + int64_t(crow) * A.c_in.ld, kcw4);
            crow = crow + 1 == Rh ? 0 : crow + 1;
        };

        Pair w[RR];
        float hf[RH];
        Pair uh[RC];
#pragma unroll
        for (int r = 0; r < RR; ++r) w[r] = Pair{0.f, 0.f};
#pragma unroll
        for (int r = 0; r < RH; ++r) hf[r] = 0.f;
#pragma unroll
        for (int r = 0; r < RC; ++r) uh[r] = Pair{0.f, 0.f};

        // block 0 staged now, block 1 in flight
        stage_load(S2);
        stage_store();
        lds_sync();
        stage_load(S2 + VB);
#pragma unroll
        for (int p = 0; p < PFH; ++p) {
            load_h(hq[p]);
            load_c(cq[p]);
        }
        static_assert(U % PFH == 0, "prefetch ring");
        for (int n0 = 0; n0 < NS; n0 += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int n = n0 + u;
                const int nb_ = n / VB, ni = n - nb_ * VB;
                if (ni == 0 && nb_ > 0) {
                    // block nb_ (loaded one block ago) replaces block nb_ - 1;
                    // block nb_ + 1 goes out
                    lds_sync();
                    stage_store();
                    lds_sync();
                    stage_load(S2 + (nb_ + 1) * VB);
                }
                // compact row n onto the checkerboard (image rows 2n, 2n + 1)
                {
                    Pair& E = w[rslot(2 * u)];
                    Pair& O = w[rslot(2 * u + 1)];
                    E.x = s2 * T[lane * VLD + ni];
                    const Pair& H = hq[u % PFH];
                    const float hx = qin ? __fmul_rn(float(__builtin_bit_cast(int, H.x)), d1) : H.x;
                    const float hy = qin ? __fmul_rn(float(__builtin_bit_cast(int, H.y)), d0) : H.y;
                    E.y = s0 * hy;
                    O.x = s1 * hx;
                    O.y = s3 * T[(64 + lane) * VLD + ni];
                }
                float cv = cq[u % PFH];
                if (lin) {
                    // the lowpass dequantised as ct_dequantize does
                    const float w = __fmul_rn(float(__builtin_bit_cast(int, cv)), l_step);
                    cv = __fadd_rn(l_mn, __fmul_rn(w, l_r));
                }
                load_h(hq[u % PFH]);
                load_c(cq[u % PFH]);
                // tree level 2 (q < 4) then level 1, step q on rows 2n - 1 - q, 2n - q
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int st = q & 3;
                    const float cf = 0.5f * A.L.c[st];
                    const int par = (FO + st) & 1;
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        const int rel = 2 * u - 1 - q + j;
                        const int rpar = (((-1 - q + j) % 2) + 2) % 2;
                        Pair& X = w[rslot(rel)];
                        const Pair& Up = w[rslot(rel - 1)];
                        const Pair& Dn = w[rslot(rel + 1)];
                        if (q < 4) {
                            if (par == 0)
                                X.x = fmaf(cf, (Up.y + from_prev(Dn.y)) - (Dn.y + from_prev(Up.y)), X.x);
                            else
                                X.y = fmaf(cf, (from_next(Up.x) + Dn.x) - (from_next(Dn.x) + Up.x), X.y);
                        } else {
                            if (rpar == par) X.x = fmaf(cf, (X.y + from_prev(X.y)) - (Dn.x + Up.x), X.x);
                            else X.y = fmaf(cf, (from_next(X.x) + X.x) - (Dn.y + Up.y), X.y);
                        }
                    }
                }
                // bandpass rows 2n - 8, 2n - 7 are final: their horizontal lowpass
                hf[hslot(2 * u - 8)] = row_lowpass<LO_R>(A.lo, w[rslot(2 * u - 8)].x, w[rslot(2 * u - 8)].y);
                hf[hslot(2 * u - 7)] = row_lowpass<LO_R>(A.lo, w[rslot(2 * u - 7)].x, w[rslot(2 * u - 7)].y);
                // lowpass row n - 6: c' = c - vertical lowpass of hf rows 2n - 12 +- LO_R
                float h[2 * LO_R + 1];
#pragma unroll
                for (int k = 0; k <= 2 * LO_R; ++k) h[k] = hf[hslot(2 * u - 12 - LO_R + k)];
                const float cp = cv - col_lowpass<LO_R>(A.lo, h);
                uh[cslot(u - 6)] = row_upsample<UP_R>(A.up, cp);
                // image rows 2m, 2m + 1 with m = n - 8
                {
                    const Pair um2 = uh[cslot(u - 10)], um1 = uh[cslot(u - 9)], u0 = uh[cslot(u - 8)];
                    const Pair up1 = uh[cslot(u - 7)], up2 = uh[cslot(u - 6)];
                    const Pair de = w[rslot(2 * u - 16)], dod = w[rslot(2 * u - 15)];
                    float ex = A.up.t[0] * u0.x, ey = A.up.t[0] * u0.y;
                    ex = fmaf(A.up.t[2], um1.x + up1.x, ex);
                    ey = fmaf(A.up.t[2], um1.y + up1.y, ey);
                    if (UP_R >= 4) {
                        ex = fmaf(A.up.t[4], um2.x + up2.x, ex);
                        ey = fmaf(A.up.t[4], um2.y + up2.y, ey);
                    }
                    float ox = A.up.t[1] * (u0.x + up1.x), oy = A.up.t[1] * (u0.y + up1.y);
                    ox = fmaf(A.up.t[3], um1.x + up2.x, ox);
                    oy = fmaf(A.up.t[3], um1.y + up2.y, oy);
                    const int r = 2 * S2 + 2 * n - LAG;          // image row of de
                    auto put = [&](int row, float a, float c) __attribute__((always_inline)) {
                        float* rp = xo + int64_t(row) * A.x_out.ld;
                        if (pair_st) {
                            // even output width: a lane stores both columns or none
                            const float v[2] = {a, c};
                            if (st0) st_vec<2>(rp, j4, v);
                        } else {
                            if (st0) st_at(rp, j4, a);
                            if (st1) st_at(rp, j4 + 4u, c);
                        }
                    };
                    if (r >= rb && r < re && r < oh) put(r, de.x + ex, de.y + ey);
                    if (r + 1 >= rb && r + 1 < re && r + 1 < oh) put(r + 1, dod.x + ox, dod.y + oy);
                }
            }
        }
    }
};

}  // namespace stream
}  // namespace ct

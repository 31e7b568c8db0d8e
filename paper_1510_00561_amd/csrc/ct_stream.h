// Register-streaming form of the deeper DFB tree levels (t >= 3), one tree
// level or two consecutive ones per pass.
//
// Every wavefront owns one strip of 128 sheared columns (two adjacent
// columns per lane) of one parent channel and streams down a block of its
// rows. Rows live in a ring of registers; a lifting step on a row reads its
// vertical neighbours from the ring and its horizontal neighbours from the
// adjacent lanes (DPP wavefront shifts). Each row is read from HBM once and
// written once; no LDS and no barriers are used.
//
// Every multiply-add is an explicit fmaf and the library is built without
// FMA contraction, so the arithmetic does not depend on the driver (per-stage
// kernel or batched group kernel). In the sheared frame Q[i, k] = P[i, k - a i] of a parent with shear a:
//   level t    : N = Q[i-1][k+1] + Q[i+1][k-1] - Q[i-1][k] - Q[i+1][k]
//   level t + 1: even rows N = Q[i-2][k+2] + Q[i+2][k-2] - Q[i-2][k+1] - Q[i+2][k-1]
//                odd rows  N = Q[i-2][k+1] + Q[i+2][k-1] - Q[i-2][k]   - Q[i+2][k]
// (all halved), step s updating rows of class (first_odd + s) & 1, where the
// class is i & 1 at level t and (i >> 1) & 1 at level t + 1.
//
// Pipeline. Rows arrive four at a time (a superstep). Step number q of the
// pass has a fixed lag L_q (in rows behind the newest loaded row): L_q =
// L_{q-1} + d_q with d_q the step's row reach (1 or 2), so when a superstep
// runs its steps in order every neighbour a step reads has already received
// the previous step. A row is final TL = sum d_q rows behind the newest one.
// Halo: TL rows above and below a block and TL columns on each side of a
// strip are loaded but not stored.
#pragma once

#include "ct_quant_stages.h"
#include "ct_stages.h"

#include <math.h>

namespace ct {
namespace stream {

// lane l receives lane l + 1's value (wavefront shift; bound_ctrl makes the
// last lane read 0, so no old value has to be set up)
__device__ __forceinline__ float from_next(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
// lane l receives lane l - 1's value (the first lane reads 0)
__device__ __forceinline__ float from_prev(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}

struct Pair {
    float x, y;   // sheared columns k0 and k0 + 1 of this lane
};

// Level-t step on row X from its upper (U) and lower (V) neighbours, or the
// odd-row level-(t+1) step with U, V two rows away.
__device__ __forceinline__ void step_near(Pair& X, const Pair& U, const Pair& V, float c) {
    const float vp = from_prev(V.y);   // V[k0 - 1]
    const float un = from_next(U.x);   // U[k0 + 2]
    X.x = fmaf(c, (U.y + vp) - (U.x + V.x), X.x);
    X.y = fmaf(c, (un + V.x) - (U.y + V.y), X.y);
}

// Even-row level-(t+1) step.
__device__ __forceinline__ void step_far(Pair& X, const Pair& U, const Pair& V, float c) {
    const float un0 = from_next(U.x), un1 = from_next(U.y);   // U[k0 + 2], U[k0 + 3]
    const float vp0 = from_prev(V.x), vp1 = from_prev(V.y);   // V[k0 - 2], V[k0 - 1]
    X.x = fmaf(c, (un0 + vp0) - (U.y + vp1), X.x);
    X.y = fmaf(c, (un1 + vp1) - (un0 + V.x), X.y);
}

__device__ __forceinline__ int pmod(int i, int n) {
    const int r = i % n;
    return r < 0 ? r + n : r;
}

// Accesses at a wave-uniform base plus a 32-bit per-lane byte offset: the
// address form with the base in scalar registers and the offset in one
// vector register, so no per-lane 64-bit address arithmetic is needed.
template <class T>
__device__ __forceinline__ T ld_at(const T* base, uint32_t byte_off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <class T>
__device__ __forceinline__ void st_at(T* base, uint32_t byte_off, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

template <int LEVELS, bool ANA, int NT>
struct StreamSplit {
    static constexpr int WAVES = NT / 64;
    static constexpr int TL = stream_halo(LEVELS);         // total lag = halo rows = halo columns
    static constexpr int HC = TL;
    static constexpr int VW = stream_cols(LEVELS);         // stored columns per strip
    // ring rows (multiple of 4): the rows the steps still read, plus two
    // supersteps of prefetched rows
    static constexpr int RING = LEVELS == 1 ? 20 : 28;
    static constexpr int UNROLL = RING / 4;
    static constexpr int NSTEP = 4 * LEVELS;

    const SplitArgs& A;
    int batch;
    Lift lift;
    __device__ StreamSplit(const SplitArgs& a, int b, const Lift& L) : A(a), batch(b), lift(L) {}

    __device__ int items() const { return stream_items(A, batch, LEVELS); }
    __device__ int tiles() const { return (items() + WAVES - 1) / WAVES; }

    // Step q of the pass: row reach d, lag, coefficient index and whether it
    // belongs to level t + 1 (class (i >> 1) & 1 and the far stencil on even
    // rows).
    struct StepInfo {
        int d, lag, s;
        bool deep;
    };
    static constexpr StepInfo info(int q) {
        if (LEVELS == 1) return StepInfo{1, q + 1, q, false};
        if (ANA) return q < 4 ? StepInfo{1, q + 1, q, false} : StepInfo{2, 4 + 2 * (q - 3), q - 4, true};
        return q < 4 ? StepInfo{2, 2 * (q + 1), q, true} : StepInfo{1, 8 + (q - 3), q - 4, false};
    }
    static constexpr int slot(int rel) { return ((rel % RING) + RING) % RING; }

    // QUANT must match A.q.idx != nullptr (the launcher picks the kernel).
    template <bool QUANT>
    __device__ __forceinline__ void run_tile(int tile) const {
        const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
        const int item = tile * WAVES + wave;
        if (item >= items()) return;
        if (lift.first_odd) run<1, QUANT>(item);
        else run<0, QUANT>(item);
    }

    // QUANT: the final subbands are indices (analysis: quantised on store,
    // synthesis: dequantised on load) with the quantiser's arithmetic.
    template <int FO, bool QUANT>
    __device__ __forceinline__ void run(int item) const {
        const StreamCounts cnt = stream_counts(A, LEVELS);
        const int nh = cnt.nh, ih = cnt.ih, iv = cnt.iv, sh = cnt.sh, sv = cnt.sv;
        const int per_plane = nh * (ih + iv);
        const int b = item / per_plane;
        int rem = item - b * per_plane;
        int pp, strip, blk;
        if (rem < nh * ih) {
            pp = rem / ih;
            rem -= pp * ih;
            blk = rem / sh;
            strip = rem - blk * sh;
        } else {
            rem -= nh * ih;
            const int v = rem / iv;
            pp = nh + v;
            rem -= v * iv;
            blk = rem / sv;
            strip = rem - blk * sv;
        }
        const stage::SplitGeom g = stage::split_geom(A, pp);
        const int nr = g.nr, nc = g.nc;
        const int kb = strip * VW, rb = blk * A.bh;
        const int ke = min(kb + VW, nc), re = min(rb + A.bh, nr);
        const int lane = threadIdx.x & 63;
        // byte offsets of the lane's two columns modulo the row, relative to
        // the row's column base (kb - HC - a i) mod nc
        const uint32_t ncb = 4u * uint32_t(nc);
        const uint32_t m0 = 4u * uint32_t(pmod(2 * lane, nc)), m1 = 4u * uint32_t(pmod(2 * lane + 1, nc));
        const int kl = kb - HC + 2 * lane;
        const bool st0 = kl >= kb && kl < ke, st1 = kl + 1 >= kb && kl + 1 < ke;
        const int S = rb - TL;                      // first loaded row (S = 0 mod 4)
        const int E = S - TL;                       // row leaving the pipeline at superstep 0
        const int NS = (re - rb + 3) / 4 + TL / 2;  // supersteps that matter
        const int t = A.t;
        const int a4b = 4 * pmod(4 * g.a, nc);      // column-base drift per superstep (bytes)
        const int r4 = 4 % nr;                      // row advance per superstep modulo nr

        const float* src = A.parent ? A.parent + b * A.parent_plane : nullptr;
        float* dst = A.child ? A.child + b * A.child_plane : nullptr;
        int16_t* qplane = QUANT ? A.q.idx + b * A.q.plane : nullptr;
        const float* qsteps = QUANT ? A.q.steps + int64_t(b) * A.q.steps_stride : nullptr;
        const int64_t cs1 = A.plane_elems >> t;          // child channel size (one level)
        const int64_t cs2 = A.plane_elems >> (t + 1);    // grandchild channel size

        // Row r of a superstep is S + 4 n + r (loads) or E + 4 n + r
        // (stores): r equals the row index modulo 4, which fixes the child
        // channel it belongs to.
        int lrow[4], lcb[4], scb[4];
        const float* lbase[4];
        float* sbase[4];
        float lsc[4], ssc[4];
        int16_t* qbase[4];        // QUANT: indices of the final subband of row class r
        float qstep[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            lrow[r] = pmod(S + r, nr);
            lcb[r] = 4 * pmod(kb - HC - g.a * (S + r), nc);
            scb[r] = 4 * pmod(kb - HC - g.a * (E + r), nc);
            int pos = 0;
            if (LEVELS == 1) pos = (r & 1) ? g.odd_pos : g.even_pos;
            else pos = stage::grandchild_pos(g.vertical, pp, r);
            const float sc = A.use_scale ? A.scale[pos] : 1.f;
            const int64_t cs = LEVELS == 1 ? cs1 : cs2;
            if (ANA) {
                lbase[r] = src + g.parent_off;
                lsc[r] = 1.f;
                sbase[r] = dst ? dst + pos * cs : nullptr;
                ssc[r] = sc;
            } else {
                lbase[r] = src ? src + pos * cs : nullptr;
                lsc[r] = sc;
                sbase[r] = dst + g.parent_off;
                ssc[r] = 1.f;
            }
            qbase[r] = QUANT ? qplane + pos * cs : nullptr;
            qstep[r] = QUANT ? qsteps[A.q.sub0 + pos] : 1.f;
        }
        const bool store_float = !ANA || !QUANT || dst != nullptr;
        // rows of the arrays that hold the superstep's rows: parents are
        // addressed by the row itself, children by row >> 1, grandchildren
        // by row >> 2
        constexpr int CSH = LEVELS == 1 ? 1 : 2;
        constexpr int LSH = ANA ? 0 : CSH;
        constexpr int SSH = ANA ? CSH : 0;

        Pair w[RING];
#pragma unroll
        for (int r = 0; r < RING; ++r) w[r] = Pair{0.f, 0.f};

        auto load4 = [&](int u_next) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const char* rp = (!ANA && QUANT) ? nullptr
                                 : reinterpret_cast<const char*>(lbase[r] + int64_t(lrow[r] >> LSH) * nc);
                uint32_t o0 = uint32_t(lcb[r]) + m0, o1 = uint32_t(lcb[r]) + m1;
                o0 = min(o0, o0 - ncb);
                o1 = min(o1, o1 - ncb);
                Pair& X = w[slot(4 * u_next + r)];
                if (!ANA && QUANT) {
                    // dequantise on load: (q * step) * scale, as ct_dequantize
                    // followed by a float load would compute
                    const int16_t* qr = qbase[r] + int64_t(lrow[r] >> LSH) * nc;
                    X.x = lsc[r] * __fmul_rn(float(qr[o0 >> 2]), qstep[r]);
                    X.y = lsc[r] * __fmul_rn(float(qr[o1 >> 2]), qstep[r]);
                } else {
                    X.x = lsc[r] * *reinterpret_cast<const float*>(rp + o0);
                    X.y = lsc[r] * *reinterpret_cast<const float*>(rp + o1);
                }
                lrow[r] += r4;
                lrow[r] = lrow[r] >= nr ? lrow[r] - nr : lrow[r];
                lcb[r] -= a4b;
                lcb[r] = lcb[r] < 0 ? lcb[r] + int(ncb) : lcb[r];
            }
        };
        auto store4 = [&](int u, int n) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = E + 4 * n + r;
                uint32_t o0 = uint32_t(scb[r]) + m0, o1 = uint32_t(scb[r]) + m1;
                o0 = min(o0, o0 - ncb);
                o1 = min(o1, o1 - ncb);
                scb[r] -= a4b;
                scb[r] = scb[r] < 0 ? scb[r] + int(ncb) : scb[r];
                if (i < rb || i >= re) continue;
                const Pair& X = w[slot(4 * u - TL + r)];
                const float v0 = ssc[r] * X.x, v1 = ssc[r] * X.y;
                if (store_float) {
                    char* rp = reinterpret_cast<char*>(sbase[r] + int64_t(i >> SSH) * nc);
                    if (st0) *reinterpret_cast<float*>(rp + o0) = v0;
                    if (st1) *reinterpret_cast<float*>(rp + o1) = v1;
                }
                if (ANA && QUANT) {
                    // quantise on store: round(c / step), as ct_quantize on the
                    // stored float
                    int16_t* qr = qbase[r] + int64_t(i >> SSH) * nc;
                    if (st0) qr[o0 >> 2] = qstage::to_index(__fdiv_rn(v0, qstep[r]));
                    if (st1) qr[o1 >> 2] = qstage::to_index(__fdiv_rn(v1, qstep[r]));
                }
            }
        };

        load4(0);
        load4(1);
        for (int n0 = 0; n0 < NS; n0 += UNROLL) {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                // the rows of the superstep after next go into ring slots that
                // no step of this superstep reads (two supersteps of latency
                // hiding)
                load4(u + 2);
#pragma unroll
                for (int q = 0; q < NSTEP; ++q) apply_step<FO>(w, u, q);
                store4(u, n0 + u);
            }
        }
    }

    template <int FO>
    __device__ __forceinline__ void apply_step(Pair* w, int u, int q) const {
        const StepInfo si = info(q);
        const float c = 0.5f * lift.c[si.s];
        const int cls = (FO + si.s) & 1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int rel = 4 * u - si.lag + j;       // row relative to 4 n0 (n0 = 0 mod UNROLL)
            const int m4 = ((j - si.lag) % 4 + 4) % 4; // row index mod 4 (S = 0 mod 4)
            const int rc = si.deep ? (m4 >> 1) & 1 : m4 & 1;
            if (rc != cls) continue;
            Pair& X = w[slot(rel)];
            const Pair& U = w[slot(rel - si.d)];
            const Pair& V = w[slot(rel + si.d)];
            if (si.deep && (m4 & 1) == 0) step_far(X, U, V, c);
            else step_near(X, U, V, c);
        }
    }
};

}  // namespace stream
}  // namespace ct

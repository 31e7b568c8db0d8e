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
    float x, y;   // columns k0 and k0 + 1 of this lane
};

// N adjacent sheared columns of one lane (lane l holds columns N l .. N l + N - 1).
template <int N>
struct Cols {
    float v[N];
};

// Column e of the lane's row, e in [-N, 2N): the lane's own value or that of
// the previous / next lane (the steps below only call it with constants).
template <int N>
__device__ __forceinline__ float col(const Cols<N>& a, int e) {
    if (e < 0) return from_prev(a.v[e + N]);
    if (e >= N) return from_next(a.v[e - N]);
    return a.v[e];
}

// Level-t step on row X from its upper (U) and lower (V) neighbours, or the
// odd-row level-(t+1) step with U, V two rows away:
// X[k] += c ((U[k+1] + V[k-1]) - (U[k] + V[k])).
template <int N>
__device__ __forceinline__ void step_near(Cols<N>& X, const Cols<N>& U, const Cols<N>& V, float c) {
#pragma unroll
    for (int e = 0; e < N; ++e)
        X.v[e] = fmaf(c, (col(U, e + 1) + col(V, e - 1)) - (U.v[e] + V.v[e]), X.v[e]);
}

// Even-row level-(t+1) step:
// X[k] += c ((U[k+2] + V[k-2]) - (U[k+1] + V[k-1])).
template <int N>
__device__ __forceinline__ void step_far(Cols<N>& X, const Cols<N>& U, const Cols<N>& V, float c) {
#pragma unroll
    for (int e = 0; e < N; ++e)
        X.v[e] = fmaf(c, (col(U, e + 2) + col(V, e - 2)) - (col(U, e + 1) + col(V, e - 1)), X.v[e]);
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

// N consecutive elements at a 4-byte aligned address as one access (global
// memory accesses of several dwords need only dword alignment).
template <int N, class T>
__device__ __forceinline__ void ld_vec(const T* base, uint32_t byte_off, T (&v)[N]) {
    __builtin_memcpy(v, __builtin_assume_aligned(reinterpret_cast<const char*>(base) + byte_off, 4), sizeof(T) * N);
}
template <int N, class T>
__device__ __forceinline__ void st_vec(T* base, uint32_t byte_off, const T (&v)[N]) {
    __builtin_memcpy(__builtin_assume_aligned(reinterpret_cast<char*>(base) + byte_off, 4), v, sizeof(T) * N);
}

template <int LEVELS, bool ANA, int NT>
struct StreamSplit {
    static constexpr int WAVES = NT / 64;
    static constexpr int CPL = stream_cols_per_lane();     // adjacent columns per lane
    using Row = Cols<CPL>;
    static constexpr int TL = stream_halo(LEVELS);         // total lag = halo rows = halo columns
    static constexpr int HC = TL;
    static constexpr int VW = stream_cols(LEVELS);         // stored columns per strip
    // supersteps of prefetched rows; ring rows (multiple of 4): the rows the
    // steps and stores still read (up to TL + 2 behind the superstep's first
    // row), the superstep's rows and the prefetched ones
    static constexpr int PF = 2;
    static constexpr int RING = (TL + 2 + 4 + 4 * PF + 3) / 4 * 4;
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
        // byte offsets of the lane's columns modulo the row, relative to the
        // row's column base (kb - HC - a i) mod nc, and whether the lane
        // stores them (halo columns are not stored)
        const uint32_t ncb = 4u * uint32_t(nc);
        const int kl = kb - HC + CPL * lane;
        uint32_t m[CPL];
#pragma unroll
        for (int e = 0; e < CPL; ++e) m[e] = 4u * uint32_t(pmod(CPL * lane + e, nc));
        // HC and kb are multiples of CPL, so a lane's columns are all halo or
        // all stored. Only the lane holding column ke - 1 of a row's last strip
        // can reach past ke: its extra columns lie below kb + VW, so they are
        // exact values of the row's first columns (modulo nc), which it then
        // stores once more with the same bits as the first strip.
        static_assert(HC % CPL == 0 && VW % CPL == 0, "strip geometry");
        const bool st_in = kl >= kb && kl < ke;
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

        Row w[RING];
        float lastq[2][UNROLL];      // odd row classes: the last lane's second column
#pragma unroll
        for (int r = 0; r < RING; ++r)
#pragma unroll
            for (int e = 0; e < CPL; ++e) w[r].v[e] = 0.f;

        // byte offset of column e for a row with column base cb (bytes)
        auto colofs = [&](int cb, int e) __attribute__((always_inline)) {
            const uint32_t o = uint32_t(cb) + m[e];
            return min(o, o - ncb);
        };
        // A lane's two columns are consecutive in memory unless they straddle
        // the end of the row. Row class r has a fixed column base modulo 2
        // (its base moves by 4 a columns per superstep, and the geometry keeps
        // nc even): even classes are always even-aligned, odd classes are when
        // the shear a is even. Loads decide by the class alone, at compile
        // time, because a branch around a prefetched load makes the compiler
        // wait for all loads where the paths join:
        //   even classes load the lane's pair;
        //   odd classes load the even-aligned pair holding the lane's first
        //   column and, with an odd shear, take the second column from the
        //   next lane (fix_odd, at the row's first use) and the last lane's
        //   from one wave-uniform load.
        // Stores branch on the row: the pair at once unless it straddles the
        // row end; the index loads of one-level passes likewise.
        static_assert(CPL == 2, "the pair forms below assume two columns per lane");
        bool lal[4], sal[4], qal[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            lal[r] = (lcb[r] >> 2) % CPL == 0;
            sal[r] = (scb[r] >> 2) % CPL == 0;
            // indices move CPL at once only from dword-aligned addresses
            qal[r] = (reinterpret_cast<uintptr_t>(qbase[r]) & 3) == 0;
        }
        constexpr uint32_t STRIP_BYTES = 4u * CPL * 64u;
        constexpr bool QLOAD_VEC = LEVELS == 1;   // measured: faster there, slower for pairs of levels
        const bool a_odd = (g.a & 1) != 0;          // odd row classes have an odd column base
        const uint32_t odd4 = a_odd ? 4u : 0u;
        const uint32_t c127 = 4u * uint32_t(127 % nc);   // last lane's second column, from the base
        auto load4 = [&](int u_next) __attribute__((always_inline)) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                Row& X = w[slot(4 * u_next + r)];
                const int64_t ro = int64_t(lrow[r] >> LSH) * nc;
                const int cb = lcb[r];
                if (!ANA && QUANT) {
                    // dequantise on load: (q * step) * scale, as ct_dequantize
                    // followed by a float load would compute
                    const int16_t* qr = qbase[r] + ro;
                    int16_t q[CPL];
                    if (QLOAD_VEC && lal[r] && qal[r]) {
                        ld_vec<CPL>(qr, colofs(cb, 0) >> 1, q);
                    } else {
#pragma unroll
                        for (int e = 0; e < CPL; ++e) q[e] = ld_at(qr, colofs(cb, e) >> 1);
                    }
#pragma unroll
                    for (int e = 0; e < CPL; ++e) X.v[e] = lsc[r] * __fmul_rn(float(q[e]), qstep[r]);
                } else if (r % 2 == 0) {
                    float x[CPL];
                    ld_vec<CPL>(lbase[r] + ro, colofs(cb, 0), x);
#pragma unroll
                    for (int e = 0; e < CPL; ++e) X.v[e] = lsc[r] * x[e];
                } else {
                    // raw values; fix_odd arranges and scales them
                    const float* rp = lbase[r] + ro;
                    float x[CPL];
                    ld_vec<CPL>(rp, colofs(cb, 0) - odd4, x);
                    X.v[0] = x[0];
                    X.v[1] = x[1];
                    uint32_t yb = uint32_t(cb) + c127;
                    yb = yb >= ncb ? yb - ncb : yb;
                    lastq[r >> 1][u_next % UNROLL] = ld_at(rp, yb);
                }
                lrow[r] += r4;
                lrow[r] = lrow[r] >= nr ? lrow[r] - nr : lrow[r];
                lcb[r] -= a4b;
                lcb[r] = lcb[r] < 0 ? lcb[r] + int(ncb) : lcb[r];
            }
        };
        // odd row classes, loaded as even-aligned pairs: with an odd base the
        // lane's columns are the pair's second element and the next lane's
        // first element (the last lane's comes from its own load); the scale
        // follows
        auto fix_odd = [&](int u) __attribute__((always_inline)) {
            if (!ANA && QUANT) return;
#pragma unroll
            for (int r = 1; r < 4; r += 2) {
                Row& X = w[slot(4 * u + r)];
                const float nx = from_next(X.v[0]);
                const float x0 = a_odd ? X.v[1] : X.v[0];
                const float x1 = a_odd ? (lane == 63 ? lastq[r >> 1][u % UNROLL] : nx) : X.v[1];
                X.v[0] = lsc[r] * x0;
                X.v[1] = lsc[r] * x1;
            }
        };
        auto store4 = [&](int u, int n) __attribute__((always_inline)) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = E + 4 * n + r;
                const int cb = scb[r];
                scb[r] -= a4b;
                scb[r] = scb[r] < 0 ? scb[r] + int(ncb) : scb[r];
                if (i < rb || i >= re) continue;
                const Row& X = w[slot(4 * u - TL + r)];
                const int64_t ro = int64_t(i >> SSH) * nc;
                float* fp = store_float ? sbase[r] + ro : nullptr;
                int16_t* qp = (ANA && QUANT) ? qbase[r] + ro : nullptr;
                float v[CPL];
                int16_t qv[CPL];
#pragma unroll
                for (int e = 0; e < CPL; ++e) {
                    v[e] = ssc[r] * X.v[e];
                    // quantise on store: round(c / step), as ct_quantize on
                    // the stored float
                    qv[e] = (ANA && QUANT) ? qstage::to_index(__fdiv_rn(v[e], qstep[r])) : int16_t(0);
                }
                const bool fvec = sal[r] || uint32_t(cb) + STRIP_BYTES <= ncb;
                if (st_in) {
                    if (store_float) {
                        if (fvec) {
                            st_vec<CPL>(fp, colofs(cb, 0), v);
                        } else {
#pragma unroll
                            for (int e = 0; e < CPL; ++e) st_at(fp, colofs(cb, e), v[e]);
                        }
                    }
                    if (ANA && QUANT) {
                        if (sal[r] && qal[r]) {
                            st_vec<CPL>(qp, colofs(cb, 0) >> 1, qv);
                        } else {
#pragma unroll
                            for (int e = 0; e < CPL; ++e) st_at(qp, colofs(cb, e) >> 1, qv[e]);
                        }
                    }
                }
            }
        };

#pragma unroll
        for (int p = 0; p < PF; ++p) load4(p);
        for (int n0 = 0; n0 < NS; n0 += UNROLL) {
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                // the rows of superstep u + PF go into ring slots that no step
                // of this superstep reads (PF supersteps of latency hiding)
                load4(u + PF);
                fix_odd(u);
#pragma unroll
                for (int q = 0; q < NSTEP; ++q) apply_step<FO>(w, u, q);
                store4(u, n0 + u);
            }
        }
    }

    template <int FO>
    __device__ __forceinline__ void apply_step(Row* w, int u, int q) const {
        const StepInfo si = info(q);
        const float c = 0.5f * lift.c[si.s];
        const int cls = (FO + si.s) & 1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int rel = 4 * u - si.lag + j;       // row relative to 4 n0 (n0 = 0 mod UNROLL)
            const int m4 = ((j - si.lag) % 4 + 4) % 4; // row index mod 4 (S = 0 mod 4)
            const int rc = si.deep ? (m4 >> 1) & 1 : m4 & 1;
            if (rc != cls) continue;
            Row& X = w[slot(rel)];
            const Row& U = w[slot(rel - si.d)];
            const Row& V = w[slot(rel + si.d)];
            if (si.deep && (m4 & 1) == 0) step_far(X, U, V, c);
            else step_near(X, U, V, c);
        }
    }
};

}  // namespace stream
}  // namespace ct

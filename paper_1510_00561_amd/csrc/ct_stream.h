// Register-streaming form of the deeper DFB tree levels (t >= 3), one, two or
// three consecutive tree levels per pass.
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
// kernel or batched group kernel).
//
// Frame. Let P be the parent channel (rows i, columns w, periodic) with
// shear a. Tree level t + v (v = 0, 1, 2 within a pass) acts on the rows of
// P as the single tree level acts on its own channel: row i belongs to the
// channel of class (i mod 2^v) at level t + v, and is updated in step s when
// (i >> v) & 1 == (first_odd + s) & 1, from the rows i -+ 2^v at the columns
//   N = (P[i - 2^v][w + A + 1] + P[i + 2^v][w - A - 1])
//     - (P[i - 2^v][w + A]     + P[i + 2^v][w - A]),   halved,
// with A = 2^v a + D_v(i): D_0 = 0, D_1 = 1 - (i & 1), D_2 = 3 - 2 (i & 1) -
// ((i >> 1) & 1) (the shears of the children and grandchildren: an even child
// has shear 2a + 1, an odd one 2a). The same float32 operations in the same
// order as one tree level per pass, so every grouping gives identical bits.
// A lane holds the columns of row i in the frame
//   Q[i][k] = P[i][k - a i - h(i)],  h(i) = floor(i / 2) for passes of two or
// three levels (0 for one level),
// where every stencil above reaches at most 2 columns (1 for one or two
// levels), and the dependence of a final value reaches HC = 4, 6 or 14
// columns to each side (and 4, 12 or 28 rows up and down).
//
// Pipeline. Rows arrive four at a time (a superstep). Step number q of the
// pass has a fixed lag L_q (in rows behind the newest loaded row): L_q =
// L_{q-1} + max(d_{q-1}, d_q) with d_q the step's row reach (1, 2 or 4), so
// when a superstep runs its steps in order every neighbour a step reads
// holds exactly the steps before it: the row below has received the previous
// step, and the row above has not yet received the next one (synthesis runs
// the reaches from large to small, where the larger of the two matters). A
// row is final TL = L_last rows behind the newest one. Halo: at least TL rows
// above and below a block and HC columns on each side of a strip are loaded
// but not stored.
#pragma once

#include "ct_quant_stages.h"
#include "ct_stages.h"

#include <math.h>

#include <type_traits>
#include <utility>

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

// Stencil of one step at pass level v on a row with index i = r (mod 4):
// N = (U[k + u1] + V[k + v1]) - (U[k + u2] + V[k + v2]) in the lanes' frame,
// U the row 2^v above, V the row 2^v below (the P-column terms w + A + 1,
// w - A - 1, w + A, w - A of the header, in that order).
struct Offs {
    int u1, u2, v1, v2;
};
__host__ __device__ constexpr Offs step_offsets(int v, int r, bool half_shear) {
    const int c0 = r & 1, c1 = (r >> 1) & 1;
    if (!half_shear) {
        if (v == 0) return Offs{1, 0, -1, 0};
        const int D = v == 1 ? 1 - c0 : 3 - 2 * c0 - c1;
        return Offs{D + 1, D, -D - 1, -D};
    }
    if (v == 0) return c0 == 0 ? Offs{0, -1, -1, 0} : Offs{1, 0, 0, 1};
    if (v == 1) return c0 == 0 ? Offs{1, 0, -1, 0} : Offs{0, -1, 0, 1};
    const int D = 3 - 2 * c0 - c1;
    return Offs{D - 1, D - 2, 1 - D, 2 - D};
}

// X[k] += c ((U[k + u1] + V[k + v1]) - (U[k + u2] + V[k + v2])).
template <int N>
__device__ __forceinline__ void step_at(Cols<N>& X, const Cols<N>& U, const Cols<N>& V, float c, Offs o) {
#pragma unroll
    for (int e = 0; e < N; ++e)
        X.v[e] = fmaf(c, (col(U, e + o.u1) + col(V, e + o.v1)) - (col(U, e + o.u2) + col(V, e + o.v2)), X.v[e]);
}

// f(integral_constant<int, I>) for I = 0 .. N-1: a loop whose index is a
// compile-time constant in the body (ring slots and row classes stay
// constants, so the ring stays in registers whatever the unroller decides).
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Pass level of step q (analysis runs the levels in order, synthesis in
// reverse), and the step's lag. A step on row X reads X - d and X + d. The
// row below must already hold the previous step and the row above must not
// yet hold the next one, so each lag exceeds the previous one by the larger
// of the two steps' reaches (for the analysis, whose reaches never shrink,
// that is the step's own reach).
__host__ __device__ constexpr int split_level_of(int levels, bool ana, int q) {
    return ana ? q / 4 : levels - 1 - q / 4;
}
__host__ __device__ constexpr int split_lag(int levels, bool ana, int q) {
    int lag = 0;
    for (int p = 0; p <= q; ++p) {
        const int d = 1 << split_level_of(levels, ana, p);
        const int dprev = p > 0 ? 1 << split_level_of(levels, ana, p - 1) : 0;
        lag += d > dprev ? d : dprev;
    }
    return lag;
}

template <int LEVELS, bool ANA, int NT>
struct StreamSplit {
    static constexpr int WAVES = NT / 64;
    static constexpr int CPL = stream_cols_per_lane();     // adjacent columns per lane
    using Row = Cols<CPL>;
    static constexpr bool HS = LEVELS >= 2;                // frame with h(i) = floor(i / 2)
    static constexpr int TL = split_lag(LEVELS, ANA, 4 * LEVELS - 1);   // total lag = halo rows
    static constexpr int HC = stream_halo_cols(LEVELS);    // halo columns on each side
    static constexpr int VW = stream_cols(LEVELS);         // stored columns per strip
    static constexpr int PER = stream_row_align(LEVELS);   // rows per period of the row classes
    static constexpr int TOP = (TL + PER - 1) / PER * PER; // rows loaded above a block
    static constexpr int NCH = 1 << LEVELS;                // final channels per parent
    static constexpr int DMAX = 1 << (LEVELS - 1);         // largest row reach of a step
    // supersteps of prefetched rows; ring rows (a multiple of the class
    // period): the rows the steps and stores still read (up to TL + DMAX
    // behind the superstep's first row), the superstep's rows and the
    // prefetched ones
    static constexpr int PF = 2;
    static constexpr int RING = (TL + DMAX + 4 + 4 * PF + PER - 1) / PER * PER;
    static constexpr int UNROLL = RING / 4;
    static constexpr int NSTEP = 4 * LEVELS;
    static_assert(RING % PER == 0 && (4 * UNROLL) % PER == 0, "ring slots must keep the row classes");

    const SplitArgs& A;
    int batch;
    Lift lift;
    __device__ StreamSplit(const SplitArgs& a, int b, const Lift& L) : A(a), batch(b), lift(L) {}

    __device__ __forceinline__ int items() const { return stream_items(A, batch, LEVELS); }
    __device__ __forceinline__ int tiles() const { return (items() + WAVES - 1) / WAVES; }

    // Step q of the pass: row reach d = 2^v, lag, lifting coefficient index
    // and pass level v (analysis runs the levels in order, synthesis in
    // reverse).
    struct StepInfo {
        int d, lag, s, v;
    };
    static constexpr StepInfo info(int q) {
        return StepInfo{1 << split_level_of(LEVELS, ANA, q), split_lag(LEVELS, ANA, q), q & 3,
                        split_level_of(LEVELS, ANA, q)};
    }
    static constexpr int slot(int rel) { return ((rel % RING) + RING) % RING; }
    static constexpr int cls_of(int rel) { return ((rel % PER) + PER) % PER; }
    // Whether rows i = r (mod 4) have an odd column base: (kb - HC) is even,
    // blocks start at rows that are multiples of 4, and the base of row i is
    // kb - HC - a i - h(i), so its parity is that of a r + h(r). AODD is the
    // parity of the parent's shear a.
    template <bool AODD>
    static constexpr bool odd_base(int r) { return (((AODD ? r : 0) + (HS ? r >> 1 : 0)) & 1) != 0; }

    // QUANT must match A.q.idx != nullptr and FO lift.first_odd (the
    // launcher picks the kernel).
    template <bool QUANT, int FO>
    __device__ __forceinline__ void run_tile(int tile) const {
        const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
        const int item = tile * WAVES + wave;
        if (item >= items()) return;
        // the shear's parity fixes every row's alignment: one instantiation each
        const bool aodd = (stage::split_geom(A, parent_of(item)).a & 1) != 0;
        if (aodd) run<FO, QUANT, true>(item);
        else run<FO, QUANT, false>(item);
    }

    // Parent channel of a work item (the decomposition of run()).
    __device__ __forceinline__ int parent_of(int item) const {
        const StreamCounts cnt = stream_counts(A, LEVELS);
        const int per_plane = cnt.nh * (cnt.ih + cnt.iv);
        const int rem = item % per_plane;
        return rem < cnt.nh * cnt.ih ? rem / cnt.ih : cnt.nh + (rem - cnt.nh * cnt.ih) / cnt.iv;
    }

    // Final channel of class c (row i = c mod 2^LEVELS) of parent pp: at
    // every pass level v an even child (bit v of c clear) of a horizontal
    // parent p sits at 2p + 1 and an odd one at 2p, of a vertical parent at
    // 2p and 2p + 1. So the position is 2^LEVELS pp + brev(c) (vertical) or
    // 2^LEVELS pp + 2^LEVELS - 1 - brev(c) (horizontal), brev reversing the
    // LEVELS bits of c.
    static constexpr int brev(int c) {
        int r = 0;
        for (int v = 0; v < LEVELS; ++v) r |= ((c >> v) & 1) << (LEVELS - 1 - v);
        return r;
    }

    // QUANT: the final subbands are indices (analysis: quantised on store,
    // synthesis: dequantised on load) with the quantiser's arithmetic.
    template <int FO, bool QUANT, bool AODD>
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
        // the item's coordinates are wave-uniform; saying so keeps every value
        // derived from them in scalar registers
        pp = __builtin_amdgcn_readfirstlane(pp);
        strip = __builtin_amdgcn_readfirstlane(strip);
        blk = __builtin_amdgcn_readfirstlane(blk);
        const stage::SplitGeom g = stage::split_geom(A, pp);
        const int nr = g.nr, nc = g.nc;
        const int kb = strip * VW, rb = blk * A.bh;
        const int ke = min(kb + VW, nc), re = min(rb + A.bh, nr);
        const int lane = threadIdx.x & 63;
        // byte offsets of the lane's columns modulo the row, relative to the
        // row's column base (kb - HC - a i - h(i)) mod nc, and whether the
        // lane stores them (halo columns are not stored)
        const uint32_t ncb = 4u * uint32_t(nc);
        const int kl = kb - HC + CPL * lane;
        uint32_t m[CPL];
#pragma unroll
        for (int e = 0; e < CPL; ++e) m[e] = 4u * uint32_t(pmod(CPL * lane + e, nc));
        // HC and kb are multiples of CPL, so a lane's columns are all halo or
        // all stored; columns at or past ke (a row's last strip) are exact
        // values of the row's first columns (modulo nc) and are not stored.
        static_assert(HC % CPL == 0 && VW % CPL == 0, "strip geometry");
        const bool st_in = kl >= kb && kl < ke;
        const int S = rb - TOP;                     // first loaded row (S = 0 mod PER)
        const int E = S - TL;                       // row leaving the pipeline at superstep 0
        const int NS = (re - E + 3) / 4;            // supersteps until row re - 1 is final
        const int t = A.t;
        auto hsh = [](int i) { return HS ? (i >> 1) : 0; };                  // h(i), floor
        const int a4b = 4 * pmod(4 * g.a + (HS ? 2 : 0), nc);   // column-base drift per superstep (bytes)
        const int r4 = 4 % nr;                      // row advance per superstep modulo nr

        const float* src = A.parent ? A.parent + b * A.parent_plane : nullptr;
        float* dst = A.child ? A.child + b * A.child_plane : nullptr;
        int16_t* qplane = QUANT ? A.q.idx + b * A.q.plane : nullptr;
        const float* qsteps = QUANT ? A.q.steps + int64_t(b) * A.q.steps_stride : nullptr;
        const int64_t csz = A.plane_elems >> (t + LEVELS - 1);   // final channel size

        // Loads and stores of a superstep touch rows of every residue r
        // modulo 4 (column bases drift alike for all of them); the final
        // channel of a row is its residue modulo PER, which the ring slot
        // fixes at compile time.
        int lrow[4], lcb[4], scb[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            lrow[r] = pmod(S + r, nr);
            lcb[r] = 4 * pmod(kb - HC - g.a * (S + r) - hsh(S + r), nc);
            scb[r] = 4 * pmod(kb - HC - g.a * (E + r) - hsh(E + r), nc);
        }
        // Final channel of class c (row residue modulo 2^LEVELS): position
        // pos(c) = P0 + sg brev(c) (final_pos unrolled), so its arrays are one
        // wave-uniform base plus a compile-time multiple of a signed stride.
        const int P0 = (pp << LEVELS) + (g.vertical ? 0 : NCH - 1);
        const int64_t cstride = g.vertical ? csz : -csz;
        const float* lfirst = ANA ? src + g.parent_off : (src ? src + P0 * csz : nullptr);
        float* sfirst = ANA ? (dst ? dst + P0 * csz : nullptr) : dst + g.parent_off;
        int16_t* qfirst = QUANT ? qplane + P0 * csz : nullptr;
        auto lbase = [&](int c) __attribute__((always_inline)) {
            return ANA ? lfirst : lfirst + brev(c & (NCH - 1)) * cstride;
        };
        auto sbase = [&](int c) __attribute__((always_inline)) {
            return ANA ? sfirst + brev(c & (NCH - 1)) * cstride : sfirst;
        };
        auto qbase = [&](int c) __attribute__((always_inline)) { return qfirst + brev(c & (NCH - 1)) * cstride; };
        // per final channel: the scale of the final store (analysis) or load
        // (synthesis) and the quantiser step
        float fsc[NCH], qstep[NCH], qrcp[NCH];
        int qf = 1;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int pos = P0 + (g.vertical ? brev(c) : -brev(c));
            fsc[c] = A.use_scale ? A.scale[pos] : 1.f;
            qstep[c] = QUANT ? qsteps[A.q.sub0 + pos] : 1.f;
            qf &= int(qstage::fast_step(qstep[c]));
        }
        // the same for every lane: a scalar branch per quantised value
        const bool qfast = __builtin_amdgcn_readfirstlane(qf) != 0;
#pragma unroll
        for (int c = 0; c < NCH; ++c) qrcp[c] = (ANA && QUANT && qfast) ? __fdiv_rn(1.f, qstep[c]) : 1.f;
        auto lsc = [&](int c) __attribute__((always_inline)) { return ANA ? 1.f : fsc[c & (NCH - 1)]; };
        auto ssc = [&](int c) __attribute__((always_inline)) { return ANA ? fsc[c & (NCH - 1)] : 1.f; };
        // indices move CPL at once only from dword-aligned addresses
        auto qal = [&](int c) __attribute__((always_inline)) {
            return (reinterpret_cast<uintptr_t>(qbase(c)) & 3) == 0;
        };
        const bool store_float = !ANA || !QUANT || dst != nullptr;
        // rows of the arrays that hold the superstep's rows: parents are
        // addressed by the row itself, final channels by row >> LEVELS
        constexpr int LSH = ANA ? 0 : LEVELS;
        constexpr int SSH = ANA ? LEVELS : 0;

        Row w[RING];
        float lastq[3][UNROLL];      // rows with an odd column base: the last lane's second column
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
        // the end of the row. Residue r has a fixed column base modulo 2 (the
        // base moves by 4 a + 2 h columns per superstep, and the geometry keeps
        // nc even), known at compile time from the shear's parity
        // (odd_base). Loads take their form from it, because a branch around
        // a prefetched load makes the compiler wait for all loads where the
        // paths join:
        //   even residues load the lane's pair;
        //   odd residues load the even-aligned pair holding the lane's first
        //   column, take the second column from the next lane (fix_odd, at
        //   the row's first use) and the last lane's from one wave-uniform
        //   load.
        // Stores branch on the row: the pair at once unless it straddles the
        // row end; the index loads of one-level passes likewise.
        static_assert(CPL == 2, "the pair forms below assume two columns per lane");
        bool sal[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) sal[r] = ((scb[r] >> 2) & 1) == 0;
        constexpr uint32_t STRIP_BYTES = 4u * CPL * 64u;
        constexpr bool QLOAD_VEC = LEVELS == 1;   // measured: faster there, slower for pairs of levels
        const uint32_t c127 = 4u * uint32_t(127 % nc);   // last lane's second column, from the base
        auto load4 = [&](int u_next) __attribute__((always_inline)) {
            static_for<4>([&](auto rc) __attribute__((always_inline)) {
                constexpr int r = decltype(rc)::value;
                const int c = cls_of(4 * u_next + r);
                Row& X = w[slot(4 * u_next + r)];
                const int64_t ro = int64_t(lrow[r] >> LSH) * nc;
                const int cb = lcb[r];
                if (!ANA && QUANT) {
                    // dequantise on load: (q * step) * scale, as ct_dequantize
                    // followed by a float load would compute
                    const int16_t* qr = qbase(c) + ro;
                    int16_t q[CPL];
                    if (QLOAD_VEC && !odd_base<AODD>(r) && qal(c)) {
                        ld_vec<CPL>(qr, colofs(cb, 0) >> 1, q);
                    } else {
#pragma unroll
                        for (int e = 0; e < CPL; ++e) q[e] = ld_at(qr, colofs(cb, e) >> 1);
                    }
#pragma unroll
                    for (int e = 0; e < CPL; ++e) X.v[e] = lsc(c) * __fmul_rn(float(q[e]), qstep[c & (NCH - 1)]);
                } else if (!odd_base<AODD>(r)) {
                    float x[CPL];
                    ld_vec<CPL>(lbase(c) + ro, colofs(cb, 0), x);
#pragma unroll
                    for (int e = 0; e < CPL; ++e) X.v[e] = lsc(c) * x[e];
                } else {
                    // raw values; fix_odd arranges and scales them
                    const float* rp = lbase(c) + ro;
                    float x[CPL];
                    ld_vec<CPL>(rp, colofs(cb, 0) - 4u, x);
                    X.v[0] = x[0];
                    X.v[1] = x[1];
                    uint32_t yb = uint32_t(cb) + c127;
                    yb = yb >= ncb ? yb - ncb : yb;
                    lastq[r - 1][u_next % UNROLL] = ld_at(rp, yb);
                }
                lrow[r] += r4;
                lrow[r] = lrow[r] >= nr ? lrow[r] - nr : lrow[r];
                lcb[r] -= a4b;
                lcb[r] = lcb[r] < 0 ? lcb[r] + int(ncb) : lcb[r];
            });
        };
        // rows with an odd base, loaded as even-aligned pairs: the lane's
        // columns are the pair's second element and the next lane's first
        // element (the last lane's comes from its own load); the scale follows
        auto fix_odd = [&](int u) __attribute__((always_inline)) {
            if (!ANA && QUANT) return;
            static_for<4>([&](auto rc) __attribute__((always_inline)) {
                constexpr int r = decltype(rc)::value;
                if constexpr (r > 0 && odd_base<AODD>(r)) {
                    const int c = cls_of(4 * u + r);
                    Row& X = w[slot(4 * u + r)];
                    const float nx = from_next(X.v[0]);
                    X.v[0] = lsc(c) * X.v[1];
                    X.v[1] = lsc(c) * (lane == 63 ? lastq[r - 1][u % UNROLL] : nx);
                }
            });
        };
        auto store4 = [&](int u, int n) __attribute__((always_inline)) {
            static_for<4>([&](auto rc) __attribute__((always_inline)) {
                constexpr int r = decltype(rc)::value;
                const int i = E + 4 * n + r;
                const int c = cls_of(4 * u - TL + r);
                const int cb = scb[r];
                scb[r] -= a4b;
                scb[r] = scb[r] < 0 ? scb[r] + int(ncb) : scb[r];
                if (i < rb || i >= re) return;
                const Row& X = w[slot(4 * u - TL + r)];
                const int64_t ro = int64_t(i >> SSH) * nc;
                float* fp = store_float ? sbase(c) + ro : nullptr;
                int16_t* qp = (ANA && QUANT) ? qbase(c) + ro : nullptr;
                float v[CPL];
                int16_t qv[CPL];
#pragma unroll
                for (int e = 0; e < CPL; ++e) {
                    v[e] = ssc(c) * X.v[e];
                    // quantise on store: round(c / step), as ct_quantize on
                    // the stored float
                    qv[e] = (ANA && QUANT) ? qstage::index_of(v[e], qstep[c & (NCH - 1)], qrcp[c & (NCH - 1)], qfast)
                                           : int16_t(0);
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
                        if (sal[r] && qal(c)) {
                            st_vec<CPL>(qp, colofs(cb, 0) >> 1, qv);
                        } else {
#pragma unroll
                            for (int e = 0; e < CPL; ++e) st_at(qp, colofs(cb, e) >> 1, qv[e]);
                        }
                    }
                }
            });
        };

        // one superstep; u is a compile-time constant (every ring slot and
        // row class is then fixed, so the ring stays in registers)
        auto superstep = [&](auto uc, int n0) __attribute__((always_inline)) {
            constexpr int u = decltype(uc)::value;
            // the rows of superstep u + PF go into ring slots that no step
            // of this superstep reads (PF supersteps of latency hiding)
            load4(u + PF);
            fix_odd(u);
            static_for<NSTEP>([&](auto qc) __attribute__((always_inline)) {
                apply_step<FO, decltype(qc)::value>(w, u);
            });
            store4(u, n0 + u);
        };
#pragma unroll
        for (int p = 0; p < PF; ++p) load4(p);
        for (int n0 = 0; n0 < NS; n0 += UNROLL) each_superstep(superstep, n0, std::make_integer_sequence<int, UNROLL>{});
    }

    template <class F, int... U>
    __device__ __forceinline__ static void each_superstep(F& f, int n0, std::integer_sequence<int, U...>) {
        (f(std::integral_constant<int, U>{}, n0), ...);
    }

    template <int FO, int Q>
    __device__ __forceinline__ void apply_step(Row* w, int u) const {
        constexpr StepInfo si = info(Q);
        const float c = 0.5f * lift.c[si.s];
        constexpr int cls = (FO + si.s) & 1;
        static_for<4>([&](auto jc) __attribute__((always_inline)) {
            constexpr int j = decltype(jc)::value;
            const int rel = 4 * u - si.lag + j;       // row relative to S + 4 n0 (both = 0 mod PER)
            const int rc = cls_of(rel);               // row index modulo PER
            if (((rc >> si.v) & 1) != cls) return;
            Row& X = w[slot(rel)];
            const Row& U = w[slot(rel - si.d)];
            const Row& V = w[slot(rel + si.d)];
            step_at(X, U, V, c, step_offsets(si.v, rc & 3, HS));
        });
    }
};

}  // namespace stream
}  // namespace ct

// Full-search block-matching motion estimation for gfx950 (paper section
// 3.2): for each 16 x 16 block of the current luminance plane, the sum of
// squared differences against every block of the previous plane displaced by
// at most w pixels, and the displacement of the smallest.
//
// One wavefront per block, four blocks per workgroup, mapped
// XCD-contiguously. The wavefront stages its block and the (16 + 2w)^2
// search window of the previous plane in LDS as 16-bit integers (4 Y, on
// the 8-bit scale: exact for the quarter-integer luminance of the YCoCg
// front end), each window row twice: as pairs starting at even columns and
// as pairs starting at odd ones, so that a candidate at any column offset
// reads aligned pairs. Each lane then takes tasks l, l + 64, ...: two
// candidates on one row offset, two columns apart, sharing their window
// reads, and accumulates their squared differences two pixels at a time: one packed
// 16-bit subtraction and one 16-bit dot product with 32-bit accumulation per
// pair (exact: at most 256 * 1020^2 < 2^31). The block's row of 16 pixels
// is a wave-uniform LDS broadcast. The winner is the smallest 64-bit key
// (sum, |dy| + |dx|, dy, dx), reduced across the wavefront.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ct_kernels.h"
#include "ct_motion.h"

namespace ct {
namespace {

constexpr int NT = 256;
constexpr int kWaves = NT / 64;
constexpr int kB = kMotionBlock;          // 16
constexpr int kPairs = kB / 2;            // pairs per block row

typedef short s2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t quarter(float v) {
    float q = rintf(v * 4.0f);
    q = fminf(fmaxf(q, 0.0f), 1020.0f);
    return uint32_t(q);
}

__device__ __forceinline__ int ssd_pair(uint32_t a, uint32_t b, int acc) {
    const s2 d = __builtin_bit_cast(s2, a) - __builtin_bit_cast(s2, b);
    return __builtin_amdgcn_sdot2(d, d, acc, false);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sums of squared differences of two candidates on one window row offset
// and two columns apart (same column parity), which share their window
// reads: `ref` is the window copy of that parity, the first candidate's row
// `rr0` and pair `k0`; the second reads pairs k0 + 1 .. k0 + 8. `cur` holds
// the block's pairs (row r at 8 r), `rp` is the window's row pitch in pairs.
// ROWS > 0 fixes the row count (full blocks); with MASK, mask[k] keeps only
// the block's own columns of pair k. Two accumulators per candidate keep the
// dot products of a row independent (integer sums: the order does not
// matter).
template <bool MASK, int ROWS>
__device__ __forceinline__ void candidate_pair_ssd(const uint32_t* cur, const uint32_t* ref,
                                                   int rr0, int k0, int rp, int bh,
                                                   const uint32_t* mask, int& sa, int& sb) {
    int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
    const int rows = ROWS > 0 ? ROWS : bh;
#pragma unroll 2
    for (int r = 0; r < rows; ++r) {
        const uint32_t* rw = ref + (rr0 + r) * rp + k0;
        uint32_t rv[kPairs + 1];
#pragma unroll
        for (int k = 0; k <= kPairs; ++k) rv[k] = rw[k];
        const uint4 c0 = *reinterpret_cast<const uint4*>(cur + kPairs * r);
        const uint4 c1 = *reinterpret_cast<const uint4*>(cur + kPairs * r + 4);
        const uint32_t c[kPairs] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
        for (int k = 0; k < kPairs; ++k) {
            uint32_t cv = c[k], va = rv[k], vb = rv[k + 1];
            if (MASK) {
                cv &= mask[k];
                va &= mask[k];
                vb &= mask[k];
            }
            if (k & 1) {
                a1 = ssd_pair(cv, va, a1);
                b1 = ssd_pair(cv, vb, b1);
            } else {
                a0 = ssd_pair(cv, va, a0);
                b0 = ssd_pair(cv, vb, b0);
            }
        }
    }
    sa = a0 + a1;
    sb = b0 + b1;
}

__device__ __forceinline__ uint64_t match_key(int ssd, int dy, int dx, int w) {
    return (uint64_t(uint32_t(ssd)) << 32) | (uint64_t(abs(dy) + abs(dx)) << 16) |
           (uint64_t(dy + w) << 8) | uint64_t(dx + w);
}

__global__ __launch_bounds__(NT) void motion_search_kernel(MotionArgs a) {
    extern __shared__ __align__(16) uint32_t smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int item = xcd_remap(blockIdx.x, gridDim.x) * kWaves + wave;
    if (item >= a.items) return;   // whole wavefront: no workgroup barrier below
    const int per_plane = a.nby * a.nbx;
    const int b = item / per_plane, rem = item - b * per_plane;
    const int by = rem / a.nbx, bx = rem - by * a.nbx;
    const int y0 = by * kB, x0 = bx * kB;
    const int bh = min(kB, a.H - y0), bw = min(kB, a.W - x0);
    const int w = a.w, S = kB + 2 * w, rp = a.rp;
    uint32_t* even = smem + wave * a.lds_per_wave;      // pair k = columns 2k, 2k + 1
    uint32_t* odd = even + a.odd_off;                    // pair k = columns 2k + 1, 2k + 2
    uint32_t* cur = even + a.cur_off;                    // block pairs, 8 per row
    const float* prev = a.prev + int64_t(b) * a.H * a.W;
    const float* curp = a.cur + int64_t(b) * a.H * a.W;

    // Search window: row r is previous-plane row y0 - w + r, column c is
    // x0 - w + c. A load covers 64 / S rows (lane l: row l / S, column l % S);
    // eight loads are issued before any is used, from addresses clamped into
    // the frame (no branch around a load, so all eight stay in flight), and
    // values outside the frame become 0.
    const int rpi = 64 / S, lr = lane / S, lc = lane - lr * S;
    const bool lane_on = lr < rpi;
    const int iters = (S + rpi - 1) / rpi;
    for (int i0 = 0; i0 < iters; i0 += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int r = (i0 + j) * rpi + lr;
            const int gy = min(max(y0 - w + r, 0), a.H - 1), gx = min(max(x0 - w + lc, 0), a.W - 1);
            v[j] = prev[gy * a.W + gx];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int r = (i0 + j) * rpi + lr, gy = y0 - w + r, gx = x0 - w + lc;
            const bool on = lane_on && r < S;
            const uint32_t q = on && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W ? quarter(v[j]) : 0u;
            uint32_t q1 = __shfl_down(q, 1);
            if (lc + 1 >= S) q1 = 0;
            if (on) {
                if ((lc & 1) == 0) even[r * rp + (lc >> 1)] = q | (q1 << 16);
                else odd[r * rp + (lc >> 1)] = q | (q1 << 16);
            }
        }
    }
    // the pad pair past each window row (read, then discarded, by the second
    // candidate of a task whose first one is the last column)
    if (lane < S) {
        even[lane * rp + S / 2] = 0;
        odd[lane * rp + S / 2] = 0;
    }
    // the block: four rows per load, lane l at row 4 i + l / 16, column l % 16
    {
        const int cx = lane & 15;
        float v[kB / 4];
#pragma unroll
        for (int i = 0; i < kB / 4; ++i) {
            const int r = min(4 * i + (lane >> 4), bh - 1);
            v[i] = curp[(y0 + r) * a.W + x0 + min(cx, bw - 1)];
        }
#pragma unroll
        for (int i = 0; i < kB / 4; ++i) {
            const int r = 4 * i + (lane >> 4);
            const uint32_t q = r < bh && cx < bw ? quarter(v[i]) : 0u;
            const uint32_t q1 = __shfl_down(q, 1);
            if ((cx & 1) == 0) cur[kPairs * r + (cx >> 1)] = q | (q1 << 16);
        }
    }
    wave_sync();

    uint32_t mask[kPairs];
    for (int k = 0; k < kPairs; ++k)
        mask[k] = 2 * k + 2 <= bw ? 0xFFFFFFFFu : (2 * k + 1 == bw ? 0x0000FFFFu : 0u);

    // Tasks: one window row offset (dy) and a column offset sc = dx + w with
    // sc mod 4 in {0, 1}, paired with sc + 2; tpr tasks per row cover every
    // sc in [0, 2w] once.
    const bool full = bh == kB && bw == kB;   // wave-uniform
    const int nt = motion_tasks(w);
    // A full block whose last pass would hold at most 32 tasks runs that pass
    // as 2 x tail half-tasks instead: lanes 2i and 2i + 1 take rows 0-7 and
    // 8-15 of task i and add their sums across the lane pair.
    int nfull, tail;
    bool split;
    motion_passes(w, full, &nfull, &tail, &split);
    const int npass = split ? nfull : (nt + 63) / 64;
    uint64_t best = ~uint64_t(0);
    auto consider = [&](bool live, int dy, int sa, int ssd_a, int ssd_b) {
        const int dxa = sa - w, dxb = sa + 2 - w;
        const bool va = live && x0 + dxa >= 0 && x0 + dxa + bw <= a.W;
        const bool vb = live && sa + 2 <= 2 * w && x0 + dxb >= 0 && x0 + dxb + bw <= a.W;
        const uint64_t ka = match_key(ssd_a, dy, dxa, w), kb = match_key(ssd_b, dy, dxb, w);
        if (va && ka < best) best = ka;
        if (vb && kb < best) best = kb;
    };
    for (int p = 0; p < npass; ++p) {
        const int t0 = 64 * p;
        int row, sa;
        motion_task(w, min(t0 + lane, nt - 1), &row, &sa);
        const int dy = row - w;
        const bool live = t0 + lane < nt && y0 + dy >= 0 && y0 + dy + bh <= a.H;
        const uint32_t* ref = (sa & 1) ? odd : even;
        int ssd_a, ssd_b;
        if (full) candidate_pair_ssd<false, kB>(cur, ref, row, sa >> 1, rp, bh, mask, ssd_a, ssd_b);
        else candidate_pair_ssd<true, 0>(cur, ref, row, sa >> 1, rp, bh, mask, ssd_a, ssd_b);
        consider(live, dy, sa, ssd_a, ssd_b);
    }
    if (split) {
        const int i = min(lane >> 1, tail - 1), h = lane & 1;
        int row, sa;
        motion_task(w, 64 * nfull + i, &row, &sa);
        const int dy = row - w;
        const bool live = (lane >> 1) < tail && y0 + dy >= 0 && y0 + dy + bh <= a.H;
        const uint32_t* ref = (sa & 1) ? odd : even;
        int ssd_a, ssd_b;
        candidate_pair_ssd<false, kB / 2>(cur + kPairs * (kB / 2) * h, ref, row + (kB / 2) * h,
                                          sa >> 1, rp, bh, mask, ssd_a, ssd_b);
        ssd_a += __shfl_xor(ssd_a, 1);
        ssd_b += __shfl_xor(ssd_b, 1);
        consider(live, dy, sa, ssd_a, ssd_b);
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const uint64_t o = __shfl_xor(best, off);
        best = o < best ? o : best;
    }
    if (lane == 0) {
        const int dy = int((best >> 8) & 0xFF) - w, dx = int(best & 0xFF) - w;
        a.mv[2 * int64_t(item)] = int16_t(dy);
        a.mv[2 * int64_t(item) + 1] = int16_t(dx);
        if (a.ssd) a.ssd[item] = int32_t(best >> 32);
    }
}

}  // namespace

// The window rows hold S / 2 + 1 pairs (the last one a zero pad). At w = 8
// (the paper's setting) the rows are padded to 21 pairs and the odd copy
// starts one word later, which halves the bank conflicts of the candidates'
// window reads (the lanes of a wavefront read pairs two apart on up to eight
// window rows); other ranges keep the dense layout.
void motion_layout(MotionArgs* a) {
    const int S = kB + 2 * a->w;
    const bool tuned = a->w == 8;
    a->rp = S / 2 + 1 + (tuned ? 4 : 0);
    a->odd_off = S * a->rp + (tuned ? 1 : 0);
    a->cur_off = (a->odd_off + S * a->rp + 3) & ~3;   // 16-byte aligned block rows
    a->lds_per_wave = a->cur_off + kPairs * kB;
}

hipError_t launch_motion_search(const MotionArgs& a, hipStream_t st) {
    const unsigned blocks = unsigned((a.items + kWaves - 1) / kWaves);
    const size_t lds = size_t(kWaves) * a.lds_per_wave * sizeof(uint32_t);
    motion_search_kernel<<<blocks, NT, lds, st>>>(a);
    return hipGetLastError();
}

}  // namespace ct

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
// reads aligned pairs. Each lane then takes candidates l, l + 64, ... and
// accumulates its squared differences two pixels at a time: one packed
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

// Sum of squared differences of one candidate; `cur` holds the block's
// pairs (row r at 8 r), `ref` the window copy whose pair `k0` starts at the
// candidate's first column, `rp` the window's row pitch in pairs. ROWS > 0
// fixes the row count (full blocks); with MASK, mask[k] keeps only the
// block's own columns of pair k. Four accumulators keep the dot products of
// a row independent (integer sums: the order does not matter).
template <bool MASK, int ROWS>
__device__ __forceinline__ int candidate_ssd(const uint32_t* cur, const uint32_t* ref, int rr0,
                                             int k0, int rp, int bh, const uint32_t* mask) {
    int acc[4] = {0, 0, 0, 0};
    const int rows = ROWS > 0 ? ROWS : bh;
#pragma unroll 2
    for (int r = 0; r < rows; ++r) {
        const uint32_t* rw = ref + (rr0 + r) * rp + k0;
        uint32_t rv[kPairs];
#pragma unroll
        for (int k = 0; k < kPairs; ++k) rv[k] = rw[k];
        const uint4 c0 = *reinterpret_cast<const uint4*>(cur + kPairs * r);
        const uint4 c1 = *reinterpret_cast<const uint4*>(cur + kPairs * r + 4);
        const uint32_t c[kPairs] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
#pragma unroll
        for (int k = 0; k < kPairs; ++k) {
            uint32_t cv = c[k], v = rv[k];
            if (MASK) {
                cv &= mask[k];
                v &= mask[k];
            }
            acc[k & 3] = ssd_pair(cv, v, acc[k & 3]);
        }
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
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
    const int w = a.w, S = kB + 2 * w, rp = S / 2 + 1;
    uint32_t* even = smem + wave * a.lds_per_wave;      // pair k = columns 2k, 2k + 1
    uint32_t* odd = even + S * rp;                       // pair k = columns 2k + 1, 2k + 2
    uint32_t* cur = odd + S * rp;                        // block pairs, 8 per row
    const float* prev = a.prev + int64_t(b) * a.H * a.W;
    const float* curp = a.cur + int64_t(b) * a.H * a.W;

    // search window: row r is previous-plane row y0 - w + r, lane l its column x0 - w + l
    for (int r = 0; r < S; ++r) {
        const int gy = y0 - w + r, gx = x0 - w + lane;
        uint32_t v = 0;
        if (lane < S && gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) v = quarter(prev[gy * a.W + gx]);
        uint32_t v1 = __shfl_down(v, 1);
        if (lane + 1 >= S) v1 = 0;
        const uint32_t pr = v | (v1 << 16);
        if (lane < S) {
            if ((lane & 1) == 0) even[r * rp + (lane >> 1)] = pr;
            else odd[r * rp + (lane >> 1)] = pr;
        }
    }
    // the block: four rows per pass, lane l at row 4 i + l / 16, column l % 16
    for (int i = 0; i < kB / 4; ++i) {
        const int r = 4 * i + (lane >> 4), cx = lane & 15;
        uint32_t v = 0;
        if (r < bh && cx < bw) v = quarter(curp[(y0 + r) * a.W + x0 + cx]);
        const uint32_t v1 = __shfl_down(v, 1);
        if ((cx & 1) == 0) cur[kPairs * r + (cx >> 1)] = v | (v1 << 16);
    }
    wave_sync();

    uint32_t mask[kPairs];
    for (int k = 0; k < kPairs; ++k)
        mask[k] = 2 * k + 2 <= bw ? 0xFFFFFFFFu : (2 * k + 1 == bw ? 0x0000FFFFu : 0u);

    const bool full = bh == kB && bw == kB;   // wave-uniform
    const int side = 2 * w + 1, nc = side * side;
    uint64_t best = ~uint64_t(0);
    for (int c0 = 0; c0 < nc; c0 += 64) {
        const int c = min(c0 + lane, nc - 1);
        const int dy = c / side - w, dx = c - (c / side) * side - w;
        const bool valid = c0 + lane < nc && y0 + dy >= 0 && x0 + dx >= 0 &&
                           y0 + dy + bh <= a.H && x0 + dx + bw <= a.W;
        const int sc = dx + w;                           // window column of the first pixel
        const uint32_t* ref = (sc & 1) ? odd : even;
        const int ssd = full ? candidate_ssd<false, kB>(cur, ref, dy + w, sc >> 1, rp, bh, mask)
                             : candidate_ssd<true, 0>(cur, ref, dy + w, sc >> 1, rp, bh, mask);
        const uint64_t key = (uint64_t(uint32_t(ssd)) << 32) |
                             (uint64_t(abs(dy) + abs(dx)) << 16) | (uint64_t(dy + w) << 8) |
                             uint64_t(dx + w);
        if (valid && key < best) best = key;
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

size_t motion_lds_per_wave(int w) {
    const int S = kB + 2 * w, rp = S / 2 + 1;
    return size_t(2 * S * rp + kPairs * kB);
}

hipError_t launch_motion_search(const MotionArgs& a, hipStream_t st) {
    const unsigned blocks = unsigned((a.items + kWaves - 1) / kWaves);
    const size_t lds = size_t(kWaves) * a.lds_per_wave * sizeof(uint32_t);
    motion_search_kernel<<<blocks, NT, lds, st>>>(a);
    return hipGetLastError();
}

}  // namespace ct

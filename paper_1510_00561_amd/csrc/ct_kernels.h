// Kernel parameter blocks and launch wrappers (device side of libct).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ct {

// Workgroups are dispatched round-robin over the 8 XCDs of MI355X, each with
// its own L2. This maps the hardware workgroup id to a logical tile index so
// that every XCD receives one contiguous range of tiles: neighbouring tiles,
// which share halo rows and columns, then meet in the same L2.
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_remap(int bid, int total) {
    const int x = bid % kNumXcd, slot = bid / kNumXcd;
    const int base = total / kNumXcd, rem = total % kNumXcd;
    return x * base + (x < rem ? x : rem) + slot;
}

// One-sided taps of a symmetric filter: t[0] centre, t[k] = tap at +-k.
struct Taps5 {
    float t[5];
};

// Four lifting constants; step s updates the sub-coset of parity
// (first_odd + s) & 1 from the other one.
struct Lift {
    float c[4];
    int first_odd;
};

// A 2-D strided array of planes.
struct View {
    float* p;
    int64_t plane;   // elements between planes
    int ld;          // elements between rows
};

struct CView {
    const float* p;
    int64_t plane;
    int ld;
};

// How the level-1 analysis reads beyond the real frame.
enum PadMode { kPadNone = 0, kPadReflect = 1, kPadZero = 2 };

// Output/input description of the four tree-level-2 channels, in subband
// order: [H a=-1 (coset (0,1)), H a=0 (1,0), V a=0 (0,0), V a=-1 (1,1)].
// Horizontal channels are (R/2) x (C/2) row major; vertical channels are
// stored transposed, (C/2) x (R/2).
struct Quad {
    float* p[4];
    int64_t plane;
    float scale[4];
};

// Quantiser indices of the final subbands of one LP level, written by the
// stage that produces them (encoder) or read by the stage that consumes them
// (decoder), in the coefficient layout: element e of subband s of plane b is
// idx[b * plane + e] with step steps[b * steps_stride + s]. The arithmetic is
// that of ct_quantize / ct_dequantize on the float value the stage stores or
// loads, so the fused paths give identical results.
struct QuantIO {
    int16_t* idx;            // null: the stage reads / writes float coefficients
    int64_t plane;
    const float* steps;
    int steps_stride;
    int sub0;                // subband index of the level's channel position 0
};

// One DFB tree level t >= 3 for all channels of an LP level whose image is
// R_j x C_j. Channels of a tree level are stored back to back in subband
// order; horizontal channels as (R_j / 2^(t-1)) x (C_j / 2), vertical ones
// transposed as (C_j / 2^(t-1)) x (R_j / 2).
struct SplitArgs {
    int t;              // tree level of the split (children level)
    int Rj, Cj;         // level image size
    const float* parent;
    float* child;
    int64_t plane_elems; // elements per plane in both buffers (Rj * Cj)
    int64_t parent_plane, child_plane;  // plane strides of the two buffers
    float scale[64];    // per child channel (applied on store / load)
    int use_scale;
    int bh;             // rows per streamed block (multiple of stream_row_align()), see block_rows()
    QuantIO q;          // final subbands as indices (analysis: written; synthesis: read)
};

// Rows per streamed block of a register-streaming stage. A wavefront streams
// one block, so a launch lasts at least one block's stream: the block is cut
// short enough that the `col_items` columns of items fill about two rounds
// of `slots` resident wavefronts, between min_rows and max_rows, a multiple
// of `align`.
__host__ __device__ inline int block_rows(int rows, int col_items, int slots, int min_rows,
                                          int max_rows, int align) {
    int nb = (rows + max_rows - 1) / max_rows;
    const int want = (2 * slots + col_items - 1) / col_items;
    if (want > nb) nb = want;
    int bh = (rows + nb - 1) / nb;
    bh = (bh + align - 1) / align * align;
    if (bh < min_rows) bh = min_rows;
    if (bh > max_rows) bh = max_rows;
    return bh;
}

// Work decomposition of the register-streaming split stages (one, two or
// three tree levels per pass): every wavefront stores a strip of
// stream_cols() sheared columns by SplitArgs::bh rows (a multiple of
// stream_row_align()) of one parent channel, and loads halo rows above and
// below and stream_halo_cols() columns on each side.
__host__ __device__ constexpr int stream_cols_per_lane() { return 2; }
__host__ __device__ constexpr int stream_halo_cols(int levels) { return levels == 1 ? 4 : levels == 2 ? 6 : 14; }
__host__ __device__ constexpr int stream_cols(int levels) {
    return 64 * stream_cols_per_lane() - 2 * stream_halo_cols(levels);
}
__host__ __device__ constexpr int stream_max_rows(int levels) { return levels == 2 ? 216 : 248; }
__host__ __device__ constexpr int stream_row_align(int levels) { return levels == 3 ? 8 : 4; }

// Per plane: horizontal parents first (each with `ih` items, `sh` strips
// across), then vertical ones (`iv`, `sv`).
struct StreamCounts {
    int nh, ih, iv, sh, sv;
};
__host__ __device__ inline StreamCounts stream_counts(const SplitArgs& a, int levels) {
    const int t = a.t, vw = stream_cols(levels), bh = a.bh;
    const int nrh = a.Rj >> (t - 2), nch = a.Cj >> 1;
    const int nrv = a.Cj >> (t - 2), ncv = a.Rj >> 1;
    StreamCounts c;
    c.nh = 1 << (t - 2);
    c.sh = (nch + vw - 1) / vw;
    c.sv = (ncv + vw - 1) / vw;
    c.ih = c.sh * ((nrh + bh - 1) / bh);
    c.iv = c.sv * ((nrv + bh - 1) / bh);
    return c;
}
__host__ __device__ inline int stream_items(const SplitArgs& a, int batch, int levels) {
    const StreamCounts c = stream_counts(a, levels);
    return c.nh * (c.ih + c.iv) * batch;
}

// Work decomposition of the register-streaming LP-level stages: every
// wavefront stores a strip of level_cols() image columns by `bh` rows (a
// multiple of 8, at most level_max_rows()) of one plane.
__host__ __device__ constexpr int level_cols() { return 96; }
__host__ __device__ constexpr int level_max_rows() { return 256; }
__host__ __device__ inline int level_items(int R, int C, int batch, int bh) {
    return ((C + level_cols() - 1) / level_cols()) * ((R + bh - 1) / bh) * batch;
}

hipError_t launch_dfb_split_analysis(const SplitArgs& a, Lift lift, int batch, hipStream_t s);
hipError_t launch_dfb_split_synthesis(const SplitArgs& a, Lift lift, int batch, hipStream_t s);

// Tree levels t and t+1 in one pass: parents at level t-1 -> grandchildren
// at level t+1 (stored back to back in subband order), and back.
hipError_t launch_dfb_split2_analysis(const SplitArgs& a, Lift lift, int batch, hipStream_t s);
hipError_t launch_dfb_split2_synthesis(const SplitArgs& a, Lift lift, int batch, hipStream_t s);
// Tree levels t, t+1 and t+2 in one pass.
hipError_t launch_dfb_split3_analysis(const SplitArgs& a, Lift lift, int batch, hipStream_t s);
hipError_t launch_dfb_split3_synthesis(const SplitArgs& a, Lift lift, int batch, hipStream_t s);

// Folds the mirrored padding back onto its sources (transpose of padding):
// out[r][c] = sum of in[r'][c'] over r' in {r, 2H-1-r}, c' in {c, 2W-1-c}
// restricted to [0, R) x [0, C).
hipError_t launch_pad_fold(CView in, int R, int C, View out, int H, int W, int batch,
                           hipStream_t s);

// Quantiser.
struct QuantArgs {
    const float* coeffs;
    const int16_t* idx_in;
    float* coeffs_out;
    int16_t* idx;
    float* side;
    const float* steps;
    int steps_stride;
    float* partials;         // [batch][kMaxPart][2]
    int64_t ncoef;           // coefficients per plane; plane stride of idx (and of coeffs_out)
    int64_t nq;              // elements [0, nq) of each plane are quantised (ncoef, or low_n)
    int64_t in_plane;        // plane stride of `coeffs` (ncoef, or low_n for a lowpass buffer)
    int64_t low_n;
    int nsub;
    int nparts;              // partial blocks per plane for the lowpass
    int vec8;                // ncoef % 8 == 0 and 16-byte aligned arrays: 8-wide accesses
    int sub_off[386];        // subband start offsets + end sentinel
};
// Pass 1 (per-block lowpass min/max partials) and pass 2 (indices).
hipError_t launch_lowpass_partial(const QuantArgs& a, int batch, hipStream_t s);
hipError_t launch_quantize(const QuantArgs& a, int batch, hipStream_t s);
hipError_t launch_dequantize(const QuantArgs& a, int batch, hipStream_t s);

}  // namespace ct

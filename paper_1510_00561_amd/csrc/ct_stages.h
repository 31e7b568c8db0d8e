// Argument blocks of the LP-level stages and the channel geometry of the DFB
// split stages, shared by the per-stage kernels, the group kernels of the
// batched form and the host-side chain builders.
#pragma once

#include "ct_kernels.h"

namespace ct {
namespace stage {

// LP level + DFB tree levels 1-2, analysis: src (the frame at level 1, read
// with pad_mode past src_h x src_w, or c_{j-1}) -> lowpass c_out and the four
// tree-level-2 channels `out`.
struct LevelAnaArgs {
    CView src;
    int src_h, src_w, pad_mode;
    int R, C;
    View c_out;
    Quad out;
    Taps5 lo, up;
    Lift L;
    int batch;
    int bh;                 // rows per streamed block, a multiple of 8
    QuantIO q;              // the four channels as indices (levels with 4 directions)
    // level 1 of the RGB encoder: when set, plane b is channel b % 3 (Y,
    // Co + 127, Cg + 127) of frame b / 3 of these 8-bit RGB frames
    // (src_h x src_w pixels, R, G, B interleaved), converted on load
    const uint8_t* rgb;
};

// DFB tree levels 1-2 + LP level, synthesis: the four channels `in` and the
// lowpass c_in -> x_out (rows < out_h, columns < out_w of the R x C result).
struct LevelSynArgs {
    Quad in;
    CView c_in;
    int R, C;
    View x_out;
    int out_h, out_w;
    Taps5 lo, up;
    Lift L;
    int batch;
    int bh;                 // rows per streamed block, a multiple of 8
    QuantIO q;              // the four channels as indices (levels with 4 directions)
    QuantIO lq;             // the lowpass c_in as indices (coarsest level)
    const float* side;      // [batch][2] lowpass (min, max), with lq
};

// Geometry of a parent channel at tree level t-1 (split at level t).
struct SplitGeom {
    int nr, nc;             // parent array size (vertical channels transposed)
    int a;                  // shear parameter
    bool vertical;
    int64_t parent_off;     // parent channel offset within a plane
    int even_pos, odd_pos;  // child channel positions at level t
};

__device__ __forceinline__ SplitGeom split_geom(const SplitArgs& A, int pp) {
    SplitGeom g;
    const int t = A.t;
    const int hp = 1 << (t - 2);                 // horizontal parents
    g.vertical = pp >= hp;
    const int q = 1 << (t - 3);
    if (!g.vertical) {
        g.a = pp - q;
        g.nr = A.Rj >> (t - 2);
        g.nc = A.Cj >> 1;
        g.odd_pos = 2 * pp;          // a' = 2a
        g.even_pos = 2 * pp + 1;     // a' = 2a + 1
    } else {
        g.a = q - 1 - (pp - hp);
        g.nr = A.Cj >> (t - 2);
        g.nc = A.Rj >> 1;
        g.even_pos = 2 * pp;
        g.odd_pos = 2 * pp + 1;
    }
    g.parent_off = pp * (A.plane_elems >> (t - 1));
    return g;
}

}  // namespace stage

// Per-stage launches of the LP-level stages (`lo_r` = reach of the lowpass
// filter: 4 for hbar, 3 for gbar in the transposes).
hipError_t launch_level_analysis(const stage::LevelAnaArgs& a, int lo_r, hipStream_t s);
hipError_t launch_level_synthesis(const stage::LevelSynArgs& a, int lo_r, hipStream_t s);

}  // namespace ct

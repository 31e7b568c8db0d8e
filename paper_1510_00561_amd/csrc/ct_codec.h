// Device side of the P-frame motion compensation (paper section 3.7) and the
// zero-run coder (section 3.8): argument blocks and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ct {
namespace codec {

constexpr int kMaxLevels = 6;
constexpr int kMaxDirs = 64;

// Packed-layout geometry of one plane, level by level. Level index 0 is the
// lowpass; index j = 1..J is LP level j. Every subband of a level has the
// same size; horizontal-cone subbands (k < nh) are stored row major in their
// natural rows_h x cols_h shape, vertical-cone ones transposed (natural
// rows_v x cols_v, stored cols_v x rows_v).
struct LevelTable {
    int J, R, C;
    int64_t ncoef;
    int64_t off[kMaxLevels + 2];     // first element of level index 0..J, then ncoef
    int nsub_l[kMaxLevels + 1];      // subbands per level (1 for the lowpass)
    int nh[kMaxLevels + 1];          // horizontal-cone subbands per level
    int rows_h[kMaxLevels + 1], cols_h[kMaxLevels + 1];
    int rows_v[kMaxLevels + 1], cols_v[kMaxLevels + 1];
    int lsh1_h[kMaxLevels + 1], lsh2_h[kMaxLevels + 1];   // log2 lattice steps (rows, cols)
    int lsh1_v[kMaxLevels + 1], lsh2_v[kMaxLevels + 1];
    int8_t o1[kMaxLevels + 1][kMaxDirs], o2[kMaxLevels + 1][kMaxDirs];   // lattice offsets
    int sub0[kMaxLevels + 1];        // subband index of the level's first subband
    // natural-row numbering of a plane for the zero-run coder: rows of
    // level index j start at row0[j]; each subband's rows are consecutive
    int row0[kMaxLevels + 2];
};

struct MCArgs {
    LevelTable T;
    const int16_t* cur;
    const int16_t* prev;
    const int16_t* mv;       // [batch / group][nby][nbx][2]
    int16_t* out;
    int batch, n, nby, nbx, group, inverse;
};

struct RLEArgs {
    LevelTable T;
    const int16_t* idx;      // [batch][ncoef]
    int16_t* sym;            // [batch][2 ncoef]
    int32_t* sub_off;        // [batch][nsub + 1]
    int32_t* rowcnt;         // [batch][nrows]
    int32_t* rowoff;         // [batch][nrows]
    int batch, nsub, nrows, p_frame;
};

hipError_t launch_mc(const MCArgs& a, hipStream_t s);
// three passes: symbols per natural row, per-plane offsets, symbols
hipError_t launch_rle(const RLEArgs& a, hipStream_t s);

}  // namespace codec
}  // namespace ct

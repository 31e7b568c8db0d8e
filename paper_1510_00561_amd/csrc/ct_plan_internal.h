// Host-side stage-chain builders shared by the plain entry points and the
// batched plan.
#pragma once

#include <vector>

#include "ct_batched.h"
#include "ct_internal.h"

namespace ct {

// Per-launch HIP-event timing (ct_profile_enable): a scope records an event
// on `st` when constructed and another at done(), only while profiling is on.
struct ProfScope {
    const char* name;
    double bytes, alg;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(const char* n, double by, double al, hipStream_t s);
    void done();
};

// `bytes`: compulsory bytes of the launch; `alg`: the algorithmic part of
// them (CT_PROFILED: all of them).
#define CT_PROFILED_ALG(name, bytes, alg, expr, stream)                            \
    do {                                                                           \
        ::ct::ProfScope ct_prof_scope_(name, double(bytes), double(alg), stream); \
        if ((expr) != hipSuccess) return CT_ERR_HIP;                               \
        ct_prof_scope_.done();                                                     \
    } while (0)
#define CT_PROFILED(name, bytes, expr, stream) CT_PROFILED_ALG(name, bytes, bytes, expr, stream)

// Transform modes, in the order used by build_transform_chain.
enum ChainMode { kModeForward = 0, kModeInverse = 1, kModeForwardAdjoint = 2, kModeInverseAdjoint = 3 };

// Quantiser of the fused encoder / decoder: indices [B][ncoef] and steps as
// for ct_quantize; `side` is read by the decoder.
struct FusedQuant {
    int16_t* idx;
    const float* steps;
    int steps_stride;
    const float* side;
};
// Per-LP-level tuning of the split passes, one int per level: the DFB tree
// levels per pass (bits 0-3: 1, 2 or 3) and the row-block height (bits 4-5:
// kHeightDefault, kHeightShort = aiming at twice the wavefronts, kHeightTall =
// at half of them, kHeightRows = the explicit rows of bits 8-15, in units of
// 4). Every code computes the same operations in the same order.
enum { kHeightDefault = 0, kHeightShort = 1, kHeightTall = 2, kHeightRows = 3 };
constexpr int kDefaultTune = 3;     // three tree levels per pass, default height
inline int tune_grouping(int code) { return code & 15; }
inline int tune_height(int code) { return (code >> 4) & 3; }
inline int tune_rows(int code) { return ((code >> 8) & 255) * 4; }
inline int tune_code(int grouping, int height, int rows = 0) { return grouping | (height << 4) | ((rows / 4) << 8); }
// A code the chain builder accepts (a cached value outside this is tuned again).
bool valid_tune(int code);
// The tuned codes of every LP level of g at this batch on the current device
// (kDefaultTune where nothing was tuned in this process).
void tuned_codes(const Geometry& g, int batch, int* codes /* [kMaxLevels] */);
// Tunes every LP level of g with three or more DFB tree levels (or takes the
// cached choice), using the workspace as scratch, and records the choices in
// the per-process table; codes[j - 1] receives level j's code.
int tune_geometry(const Geometry& g, int batch, char* ws, const Workspace& w, hipStream_t st, int* codes);
// With `rgb` (forward mode only) the level-1 stage reads the planes from
// 8-bit RGB frames instead of `in`: plane b is channel b % 3 of frame b / 3.
void build_transform_chain(const Geometry& g, int batch, int mode, const float* in, float* out,
                           char* ws, const Workspace& w, const int* tune,
                           std::vector<StageDesc>& chain, const FusedQuant* fq = nullptr,
                           const uint8_t* rgb = nullptr);
// Quantiser stages of the lowpass alone (fused encoder): `low` holds each
// plane's lowpass at stride `low_plane`.
int build_lowpass_quant_chain(const Geometry& g, int batch, const float* low, int64_t low_plane,
                              const float* steps, int steps_stride, int16_t* idx, float* side,
                              char* ws, const Workspace& w, std::vector<StageDesc>& chain);
int build_quant_chain(const Geometry& g, int batch, const float* coeffs, const float* steps,
                      int steps_stride, int16_t* idx, float* side, char* ws, const Workspace& w,
                      std::vector<StageDesc>& chain);
int build_dequant_chain(const Geometry& g, int batch, const int16_t* idx, const float* steps,
                        int steps_stride, const float* side, float* coeffs,
                        std::vector<StageDesc>& chain);
int launch_stage(const StageDesc& d, hipStream_t st);
int launch_chain(const std::vector<StageDesc>& chain, hipStream_t st);
// launch_chain with the level-1 split passes of a transform chain on a second
// stream beside the coarser levels (same results); CT_SERIAL_LEVELS=1 in the
// environment launches everything on `st` in chain order.
int launch_chain_forked(const std::vector<StageDesc>& chain, hipStream_t st);
int fill_quant_args(const Geometry& g, QuantArgs* a);
int resident_waves();
// Rows per streamed block of an LP-level stage and of a split stage.
int level_block_rows(int Rj, int Cj, int batch, bool synthesis);
int split_block_rows(const SplitArgs& a, int batch, int levels, int height = kHeightDefault, int rows = 0);

// Work-queue tiles of an LP-level stage (one wavefront item per strip and
// row block, kBatchedThreads / 64 per tile).
inline int level_stage_tiles(int R, int C, int batch, int bh) {
    constexpr int waves = kBatchedThreads / 64;
    return (level_items(R, C, batch, bh) + waves - 1) / waves;
}

// Work-queue tiles of a DFB split stage covering `levels` (1, 2 or 3) tree
// levels: one wavefront item per strip, kBatchedThreads / 64 per tile.
inline int split_stage_tiles(const SplitArgs& a, int batch, int levels) {
    constexpr int waves = kBatchedThreads / 64;
    return (stream_items(a, batch, levels) + waves - 1) / waves;
}

}  // namespace ct

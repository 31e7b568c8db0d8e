// Internal declarations shared by the host orchestration and the kernels.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/ct.h"

namespace ct {

// Maximum directional subbands per level and LP levels.
constexpr int kMaxDirs = 64;
constexpr int kMaxLevels = CT_MAX_LEVELS;

// Resolved geometry of one plane (host side).
struct Geometry {
    int H = 0, W = 0, J = 0;
    int filters = CT_FILTERS_CDF97;  // filter pair of the LP and the DFB
    int recon = CT_RECON_DUAL;       // LP reconstruction of the inverse
    int dirs[kMaxLevels] = {0};
    int l[kMaxLevels] = {0};         // log2 dirs
    int e = 0;                       // padding exponent
    int R = 0, C = 0;                // torus size
    int64_t ncoef = 0;
    int nsub = 0;
    int64_t level_off[kMaxLevels + 2] = {0};  // packed offset of level j's first subband
    int64_t low_n = 0;               // lowpass element count
};

// Builds and validates a Geometry; returns CT_OK or an error code.
int resolve(const ct_geom* g, Geometry* out);

// Fills the packed subband table (lowpass first, then levels J..1 in k order).
void subband_table(const Geometry& g, ct_subband* table, int cap);

// Scale exponent of every final subband of a DFB with l tree levels, in k
// order: the number of even minus odd channel choices on its path from the
// root. Lifting runs without its per-level +-zeta scaling; the product
// zeta^e is applied once where a subband is stored or loaded.
void dfb_scale_exponents(int l, int* out /* [2^l] */);

// Workspace layout for a batch (byte offsets, each 256-byte aligned).
struct Workspace {
    size_t c_off[kMaxLevels + 1] = {0};   // c_j for j = 1..J-1 ([B][R>>j][C>>j])
    size_t d_off = 0;                      // [B][R][C]
    size_t a_off = 0;                      // [B][R][C]
    size_t b_off = 0;                      // [B][R][C]
    size_t a2_off = 0, b2_off = 0;         // [B][R/2][C/2]: the channels of levels >= 2
    size_t part_off = 0;                   // quantiser partials [B][kMaxPart][2]
    size_t low_off = 0;                    // lowpass for the fused encoder [B][low_n]
    size_t total = 0;
};
constexpr int kMaxPart = 256;
Workspace workspace_layout(const Geometry& g, int batch);
// Bytes of the quantiser's lowpass partials for `batch` planes.
inline size_t quantize_partial_bytes(int batch) { return size_t(batch) * kMaxPart * 2 * sizeof(float); }
// Argument validation of ct_quantize (host only, nothing enqueued).
int check_quantize(const ct_geom* geom, int32_t batch, const float* coeffs, const float* steps,
                   int32_t steps_stride, const int16_t* idx, const float* side);
// ct_quantize with its lowpass partials in caller-given device memory of
// `partial_bytes` bytes (at least quantize_partial_bytes(batch)) in place of
// the workspace; validation and errors as for ct_quantize.
int quantize_with_partials(const ct_geom* geom, int32_t batch, const float* coeffs,
                           const float* steps, int32_t steps_stride, int16_t* idx, float* side,
                           void* partials, size_t partial_bytes, hipStream_t stream);

// Filters and lifting constants, derived at first use from the closed form
// of a filter pair: CT_FILTERS_CDF97 (the paper's 9-7 pair) or
// CT_FILTERS_LEGALL53. Shorter filters leave their outer taps and lifting
// steps zero, so that every stage runs the 9-7 stencils unchanged.
struct Constants {
    double hbar[5];   // LP analysis lowpass, unit DC: taps 0..4 (symmetric)
    double gbar[4];   // LP synthesis lowpass, sum 2: taps 0..3 (symmetric)
    double alpha, beta, gamma, delta, zeta;   // lifting factorisation
    bool ok;
};
const Constants& constants(int filters = CT_FILTERS_CDF97);

}  // namespace ct

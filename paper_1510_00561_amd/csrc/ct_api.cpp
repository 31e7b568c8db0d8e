// Exported C ABI of libct: validation and launch orchestration.
//
// Forward CT (paper section 2.1, Fig. 1; layout of section 3.3), per LP level
// j = 1..J:
//   LP analysis of c_{j-1} -> c_j (lowpass, to the next level or the packed
//   output) and d_j (bandpass, workspace);
//   DFB tree levels 1-2 on d_j -> four channels;
//   DFB tree levels 3..l_j, one sheared split per tree level, the last one
//   storing straight into the packed coefficient vector.
// The inverse runs the mirror image from level J down to 1 and crops the
// padding. The transposes reuse the same kernels: the LP stages with the two
// filters swapped, and the lifting stages with their steps reversed and
// predict/update roles exchanged.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ct_batched.h"
#include "ct_internal.h"
#include "ct_kernels.h"
#include "ct_plan_internal.h"

using namespace ct;

namespace {

enum class Mode { Forward, Inverse, ForwardAdjoint, InverseAdjoint };

Taps5 taps_h(int filters) {
    const Constants& k = constants(filters);
    Taps5 t;
    for (int i = 0; i < 5; ++i) t.t[i] = float(k.hbar[i]);
    return t;
}

Taps5 taps_g(int filters) {
    const Constants& k = constants(filters);
    Taps5 t;
    for (int i = 0; i < 4; ++i) t.t[i] = float(k.gbar[i]);
    t.t[4] = 0.f;
    return t;
}

Lift lift_for(Mode m, int filters) {
    const Constants& k = constants(filters);
    Lift L;
    switch (m) {
        case Mode::Forward:   // odd += a N(even); even += b; odd += g; even += d
            L = Lift{{float(k.alpha), float(k.beta), float(k.gamma), float(k.delta)}, 1};
            break;
        case Mode::Inverse:   // undo in reverse: even -= d; odd -= g; even -= b; odd -= a
            L = Lift{{float(-k.delta), float(-k.gamma), float(-k.beta), float(-k.alpha)}, 0};
            break;
        case Mode::ForwardAdjoint:   // transpose of forward, applied coefficients -> image
            L = Lift{{float(k.delta), float(k.gamma), float(k.beta), float(k.alpha)}, 1};
            break;
        case Mode::InverseAdjoint:   // transpose of inverse, applied image -> coefficients
        default:
            L = Lift{{float(-k.alpha), float(-k.beta), float(-k.gamma), float(-k.delta)}, 0};
            break;
    }
    return L;
}

// zeta^(sign * e_k) for the final subbands of a DFB with l tree levels
void scale_table(int l, int sign, int filters, float* out) {
    int e[kMaxDirs];
    dfb_scale_exponents(l, e);
    const double z = constants(filters).zeta;
    for (int k = 0; k < (1 << l); ++k) out[k] = float(pow(z, double(sign * e[k])));
}

bool fault_injected() {
    const char* f = getenv("CT_FAULT_INJECT");
    return f && strcmp(f, "launch") == 0;
}

}  // namespace

namespace ct {

// ------------------------------------------------------------ profiling
// Event pairs around launches, recorded only while enabled. The pool is
// created by ct_profile_enable so that recording never allocates.
struct ProfRecord {
    const char* name;
    double bytes, alg;
    hipEvent_t a, b;
};
struct Profiler {
    std::mutex mu;
    bool on = false;
    bool dropped = false;
    std::vector<hipEvent_t> pool;
    size_t next = 0;
    std::vector<ProfRecord> recs;
};
static Profiler& profiler() {
    static Profiler p;
    return p;
}

ProfScope::ProfScope(const char* n, double by, double al, hipStream_t s) : name(n), bytes(by), alg(al), st(s) {
    Profiler& p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    if (!p.on) return;
    if (p.next + 2 > p.pool.size()) {
        p.dropped = true;
        return;
    }
    a = p.pool[p.next++];
    b = p.pool[p.next++];
    hipEventRecord(a, st);
}

void ProfScope::done() {
    if (!a) return;
    Profiler& p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    hipEventRecord(b, st);
    p.recs.push_back(ProfRecord{name, bytes, alg, a, b});
}

}  // namespace ct

namespace {

int check_common(const ct_geom* geom, int32_t batch, Geometry* g) {
    if (!geom) return CT_ERR_ARG;
    if (batch < 0 || batch > 65535) return CT_ERR_ARG;
    return resolve(geom, g);
}

// Groups of DFB tree levels >= 3 run per pass: `grouping` (1, 2 or 3)
// levels per pass from the top, and the remaining levels in a last, shorter
// pass.
int split_groups(int l, int grouping, int* first, int* count) {
    int n = 0;
    for (int t = 3; t <= l;) {
        const int c = t + grouping - 1 <= l ? grouping : l - t + 1;
        first[n] = t;
        count[n] = c;
        ++n;
        t += c;
    }
    return n;
}

}  // namespace

namespace ct {

// Wavefronts of the streaming stages resident at once on the current device
// (about 150 VGPRs each: three per SIMD, four SIMDs per CU), cached per
// device.
int resident_waves() {
    static std::mutex mu;
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 3072;
    std::lock_guard<std::mutex> lock(mu);
    if (!cached[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cached[dev] = 12 * cus;
    }
    return cached[dev];
}

int level_block_rows(int Rj, int Cj, int batch, bool synthesis) {
    const int strips = (Cj + level_cols() - 1) / level_cols();
    // The synthesis streams 32 halo rows per block and runs fastest with
    // blocks about four times as tall, fewer wavefronts than slots (measured
    // at 1080p: 448 against 506 us per step, 466 at twice as tall); the
    // analysis is best at the default.
    if (synthesis) return block_rows(Rj, strips * batch, resident_waves() / 4, 32, 4 * level_max_rows(), 8);
    return block_rows(Rj, strips * batch, resident_waves(), 32, level_max_rows(), 8);
}

int split_block_rows(const SplitArgs& a, int batch, int levels, int height, int rows) {
    if (height == kHeightRows && rows > 0) {
        const int al = stream_row_align(levels);
        int bh = (rows + al - 1) / al * al;
        if (bh > stream_max_rows(levels)) bh = stream_max_rows(levels) / al * al;
        return bh;
    }
    const int t = a.t, vw = stream_cols(levels);
    const int nrh = a.Rj >> (t - 2), nch = a.Cj >> 1, nrv = a.Cj >> (t - 2), ncv = a.Rj >> 1;
    const int cols = (1 << (t - 2)) * ((nch + vw - 1) / vw + (ncv + vw - 1) / vw) * batch;
    // one-level passes carry a small halo and few instructions per row: they
    // run fastest with shorter blocks and four times as many wavefronts;
    // three-level passes with twice as many (1080p level 1: 120-row instead
    // of 240-row blocks, 318 against 338 us for the quantising analysis; three
    // and four times as many were slower). The tuner's height choice doubles
    // or halves the wavefronts aimed at.
    int slots = levels == 1 ? 4 * resident_waves() : levels == 3 ? 2 * resident_waves() : resident_waves();
    if (height == kHeightShort) slots *= 2;
    if (height == kHeightTall) slots /= 2;
    return block_rows(nrh > nrv ? nrh : nrv, cols, slots, 32, stream_max_rows(levels),
                      stream_row_align(levels));
}

// Stage type of a split pass over `levels` tree levels.
static int split_type(int levels, bool analysis, bool quant) {
    static const int ana[3] = {kStSplit1Ana, kStSplit2Ana, kStSplit3Ana};
    static const int anaq[3] = {kStSplit1AnaQ, kStSplit2AnaQ, kStSplit3AnaQ};
    static const int syn[3] = {kStSplit1Syn, kStSplit2Syn, kStSplit3Syn};
    static const int synq[3] = {kStSplit1SynQ, kStSplit2SynQ, kStSplit3SynQ};
    const int i = levels - 1;
    return analysis ? (quant ? anaq[i] : ana[i]) : (quant ? synq[i] : syn[i]);
}

// Subband index of the first subband of LP level j in the coefficient layout
// (lowpass first, then levels J..1).
static int first_subband(const Geometry& g, int j) {
    int s = 1;
    for (int i = g.J; i > j; --i) s += g.dirs[i - 1];
    return s;
}

// Stage chain of one transform direction (see ct_batched.h). `tune[j]`
// selects the DFB tree levels per split pass (1, 2 or 3) and the row-block
// height of the split passes at LP level j (tune_grouping, tune_height). With `fq`
// the final subbands are quantised where the forward transform produces
// them, or dequantised where the inverse consumes them (the fused encoder
// and decoder); the float coefficients `out` / `in` may then be null.
void build_transform_chain(const Geometry& g, int batch, int mode_i, const float* in, float* out,
                           char* ws, const Workspace& w, const int* tune,
                           std::vector<StageDesc>& chain, const FusedQuant* fq, const uint8_t* rgb) {
    const Mode mode = Mode(mode_i);
    const bool analysis = mode == Mode::Forward || mode == Mode::InverseAdjoint;
    const bool plain_filters = mode == Mode::Forward || mode == Mode::Inverse;
    const Taps5 lo = plain_filters ? taps_h(g.filters) : taps_g(g.filters);
    const Taps5 up = plain_filters ? taps_g(g.filters) : taps_h(g.filters);
    const int lo_r = plain_filters ? 4 : 3;
    const Lift L = lift_for(mode, g.filters);
    // Burt-Adelson reconstruction: the inverse's LP synthesis without the
    // correction of c, i.e. the dual-frame stage with a zero correction
    // filter (its `lo`); the transpose of that synthesis is the LP analysis
    // without the prediction, i.e. a zero `up`. Zero taps add exact zeros.
    const bool ba = g.recon == CT_RECON_BURT_ADELSON;
    const Taps5 zero{};
    const int64_t RC = int64_t(g.R) * g.C;
    float* D = reinterpret_cast<float*>(ws + w.d_off);
    // channel buffers of LP level j: level 1 has its own pair, the coarser
    // levels share a second one (a plane of it holds R C / 4 floats)
    float* const A1 = reinterpret_cast<float*>(ws + w.a_off);
    float* const B1 = reinterpret_cast<float*>(ws + w.b_off);
    float* const A2 = reinterpret_cast<float*>(ws + w.a2_off);
    float* const B2 = reinterpret_cast<float*>(ws + w.b2_off);
    auto push = [&](StageDesc d) {
        d.batch = batch;
        d.lift = L;
        d.lo_r = lo_r;
        chain.push_back(d);
    };
    if (analysis) {
        float* coeffs = out;
        for (int j = 1; j <= g.J; ++j) {
            const int Rj = g.R >> (j - 1), Cj = g.C >> (j - 1);
            StageDesc d;
            memset(&d, 0, sizeof(d));
            d.type = kStLevelAna;
            stage::LevelAnaArgs& a = d.u.la;
            if (j == 1) {
                a.src = CView{in, int64_t(g.H) * g.W, g.W};
                a.src_h = g.H;
                a.src_w = g.W;
                a.pad_mode = mode == Mode::Forward ? kPadReflect : kPadZero;
                a.rgb = mode == Mode::Forward ? rgb : nullptr;
            } else {
                a.src = CView{reinterpret_cast<const float*>(ws + w.c_off[j - 1]), int64_t(Rj) * Cj, Cj};
                a.src_h = Rj;
                a.src_w = Cj;
                a.pad_mode = kPadNone;
            }
            if (j < g.J)
                a.c_out = View{reinterpret_cast<float*>(ws + w.c_off[j]), int64_t(Rj / 2) * (Cj / 2), Cj / 2};
            else if (coeffs)
                a.c_out = View{coeffs, g.ncoef, Cj / 2};
            else    // fused encoder without float coefficients: the lowpass in the workspace
                a.c_out = View{reinterpret_cast<float*>(ws + w.low_off), g.low_n, Cj / 2};
            a.R = Rj;
            a.C = Cj;
            const int l = g.l[j - 1];
            float* const A = j == 1 ? A1 : A2;
            float* const Bf = j == 1 ? B1 : B2;
            const int64_t PS = j == 1 ? RC : RC / 4;     // plane stride of the channel buffers
            float* level = coeffs ? coeffs + g.level_off[j] : nullptr;
            const int64_t q4 = int64_t(Rj) * Cj / 4;
            const QuantIO qio = fq ? QuantIO{fq->idx + g.level_off[j], g.ncoef, fq->steps, fq->steps_stride,
                                             first_subband(g, j)}
                                   : QuantIO{nullptr, 0, nullptr, 0, 0};
            float sc[kMaxDirs];
            scale_table(l, mode == Mode::Forward ? +1 : -1, g.filters, sc);
            for (int k = 0; k < 4; ++k) {
                a.out.p[k] = l == 2 ? (level ? level + k * q4 : nullptr) : A + k * q4;
                a.out.scale[k] = l == 2 ? sc[k] : 1.f;
            }
            a.out.plane = l == 2 ? g.ncoef : PS;
            if (l == 2 && qio.idx) {
                a.q = qio;
                d.type = kStLevelAnaQ;
            }
            a.lo = lo;
            a.up = (ba && mode == Mode::InverseAdjoint) ? zero : up;
            a.L = L;
            a.batch = batch;
            a.bh = level_block_rows(Rj, Cj, batch, false);
            d.ntiles = level_stage_tiles(Rj, Cj, batch, a.bh);
            // compulsory bytes: input, lowpass, the four channels (indices
            // and / or floats when they are the final subbands)
            const double chan = l == 2 ? (level ? 4.0 : 0.0) + (qio.idx ? 2.0 : 0.0) : 4.0;
            // source bytes per pixel of a plane: a float, or (RGB encoder) the
            // frame's 3 bytes, read once for each of its three planes
            const double src_b = (j == 1 && a.rgb) ? 3.0 : 4.0;
            d.bytes = batch * (src_b * double(a.src_h) * a.src_w + 4.0 * double(Rj / 2) * (Cj / 2) +
                               chan * double(Rj) * Cj);
            // algorithmic: the frame (level 1), the float lowpass when it is
            // the caller's output, the final subbands when this stage makes them
            d.alg = batch * ((j == 1 ? (a.rgb ? 1.0 : 4.0) * double(a.src_h) * a.src_w : 0.0) +
                             (j == g.J && coeffs ? 4.0 * double(Rj / 2) * (Cj / 2) : 0.0) +
                             (l == 2 ? chan * double(Rj) * Cj : 0.0));
            push(d);
            int first[4], count[4];
            const int ng = split_groups(l, tune_grouping(tune[j - 1]), first, count);
            const int hm = tune_height(tune[j - 1]), hr = tune_rows(tune[j - 1]);
            float* cur = A;
            float* other = Bf;
            for (int gi = 0; gi < ng; ++gi) {
                const bool last = gi == ng - 1;
                StageDesc e;
                memset(&e, 0, sizeof(e));
                e.type = split_type(count[gi], true, false);
                SplitArgs& sa = e.u.sp;
                sa.t = first[gi];
                sa.Rj = Rj;
                sa.Cj = Cj;
                sa.parent = cur;
                sa.parent_plane = PS;
                sa.plane_elems = int64_t(Rj) * Cj;
                if (last) {
                    sa.child = level;
                    sa.child_plane = g.ncoef;
                    sa.use_scale = 1;
                    memcpy(sa.scale, sc, sizeof(float) * (1 << l));
                    sa.q = qio;
                    if (qio.idx) e.type = split_type(count[gi], true, true);
                } else {
                    sa.child = other;
                    sa.child_plane = PS;
                }
                sa.bh = split_block_rows(sa, batch, count[gi], hm, hr);
                e.ntiles = split_stage_tiles(sa, batch, count[gi]);
                const double out_b = last ? (level ? 4.0 : 0.0) + (qio.idx ? 2.0 : 0.0) : 4.0;
                e.bytes = batch * (4.0 + out_b) * double(Rj) * Cj;
                e.alg = last ? batch * out_b * double(Rj) * Cj : 0.0;
                push(e);
                float* tmp = cur;
                cur = other;
                other = tmp;
            }
        }
        return;
    }
    const float* coeffs = in;
    for (int j = g.J; j >= 1; --j) {
        const int Rj = g.R >> (j - 1), Cj = g.C >> (j - 1);
        const int l = g.l[j - 1];
        float* const A = j == 1 ? A1 : A2;
        float* const Bf = j == 1 ? B1 : B2;
        const int64_t PS = j == 1 ? RC : RC / 4;
        const float* level = coeffs ? coeffs + g.level_off[j] : nullptr;
        const int64_t q4 = int64_t(Rj) * Cj / 4;
        const QuantIO qio = fq ? QuantIO{const_cast<int16_t*>(fq->idx) + g.level_off[j], g.ncoef, fq->steps,
                                         fq->steps_stride, first_subband(g, j)}
                               : QuantIO{nullptr, 0, nullptr, 0, 0};
        float sc[kMaxDirs];
        scale_table(l, mode == Mode::Inverse ? -1 : +1, g.filters, sc);
        StageDesc d;
        memset(&d, 0, sizeof(d));
        d.type = kStLevelSyn;
        stage::LevelSynArgs& a = d.u.ls;
        if (l == 2) {
            for (int k = 0; k < 4; ++k) {
                a.in.p[k] = level ? const_cast<float*>(level) + k * q4 : nullptr;
                a.in.scale[k] = sc[k];
            }
            a.in.plane = g.ncoef;
            a.q = qio;
            if (qio.idx) d.type = kStLevelSynQ;
        } else {
            int first[4], count[4];
            const int ng = split_groups(l, tune_grouping(tune[j - 1]), first, count);
            const int hm = tune_height(tune[j - 1]), hr = tune_rows(tune[j - 1]);
            float* cur = A;
            float* other = Bf;
            for (int gi = ng - 1; gi >= 0; --gi) {
                StageDesc e;
                memset(&e, 0, sizeof(e));
                e.type = split_type(count[gi], false, false);
                SplitArgs& sa = e.u.sp;
                sa.t = first[gi];
                sa.Rj = Rj;
                sa.Cj = Cj;
                sa.plane_elems = int64_t(Rj) * Cj;
                sa.child = cur;             // output: the parents
                sa.child_plane = PS;
                if (gi == ng - 1) {
                    sa.parent = level;      // input: the final subbands
                    sa.parent_plane = g.ncoef;
                    sa.use_scale = 1;
                    memcpy(sa.scale, sc, sizeof(float) * (1 << l));
                    sa.q = qio;
                    if (qio.idx) e.type = split_type(count[gi], false, true);
                } else {
                    sa.parent = other;
                    sa.parent_plane = PS;
                }
                sa.bh = split_block_rows(sa, batch, count[gi], hm, hr);
                e.ntiles = split_stage_tiles(sa, batch, count[gi]);
                const double in_b = (gi == ng - 1 && qio.idx) ? 2.0 : 4.0;
                e.bytes = batch * (in_b + 4.0) * double(Rj) * Cj;
                e.alg = gi == ng - 1 ? batch * in_b * double(Rj) * Cj : 0.0;
                push(e);
                float* tmp = cur;
                cur = other;
                other = tmp;
            }
            for (int k = 0; k < 4; ++k) {
                a.in.p[k] = other + k * q4;
                a.in.scale[k] = 1.f;
            }
            a.in.plane = PS;
        }
        a.c_in = (j == g.J)
                     ? CView{coeffs, g.ncoef, Cj / 2}
                     : CView{reinterpret_cast<const float*>(ws + w.c_off[j]), int64_t(Rj / 2) * (Cj / 2), Cj / 2};
        if (j == g.J && fq) {
            // fused decoder: the lowpass indices, dequantised on load
            a.lq = QuantIO{const_cast<int16_t*>(fq->idx), g.ncoef, fq->steps, fq->steps_stride, 0};
            a.side = fq->side;
            d.type = kStLevelSynQ;
        }
        a.R = Rj;
        a.C = Cj;
        a.out_h = Rj;
        a.out_w = Cj;
        if (j == 1 && mode == Mode::Inverse) {
            a.x_out = View{out, int64_t(g.H) * g.W, g.W};
            a.out_h = g.H;
            a.out_w = g.W;
        } else if (j == 1) {
            a.x_out = View{D, RC, g.C};
        } else {
            a.x_out = View{reinterpret_cast<float*>(ws + w.c_off[j - 1]), int64_t(Rj) * Cj, Cj};
        }
        a.lo = (ba && mode == Mode::Inverse) ? zero : lo;
        a.up = up;
        a.L = L;
        a.batch = batch;
        a.bh = level_block_rows(Rj, Cj, batch, true);
        d.ntiles = level_stage_tiles(Rj, Cj, batch, a.bh);
        const double c_b = (j == g.J && fq) ? 2.0 : 4.0;
        const double ch_b = (l == 2 && fq) ? 2.0 : 4.0;
        d.bytes = batch * (c_b * double(Rj / 2) * (Cj / 2) + ch_b * double(Rj) * Cj +
                           4.0 * double(a.out_h) * a.out_w);
        // algorithmic: the lowpass (coarsest level), the final subbands when
        // this stage reads them, the frame (level 1)
        d.alg = batch * ((j == g.J ? c_b * double(Rj / 2) * (Cj / 2) : 0.0) +
                         (l == 2 ? ch_b * double(Rj) * Cj : 0.0) +
                         (j == 1 ? 4.0 * double(a.out_h) * a.out_w : 0.0));
        push(d);
    }
}

}  // namespace ct

namespace {

const char* stage_name(int type) {
    switch (type) {
        case kStLevelAna:
        case kStLevelAnaQ: return "lp_dfb12_analysis";
        case kStSplit1Ana:
        case kStSplit1AnaQ: return "dfb_split_analysis";
        case kStSplit2Ana:
        case kStSplit2AnaQ: return "dfb_split2_analysis";
        case kStSplit3Ana:
        case kStSplit3AnaQ: return "dfb_split3_analysis";
        case kStSplit3Syn:
        case kStSplit3SynQ: return "dfb_split3_synthesis";
        case kStPartial: return "lowpass_partial";
        case kStQuantize: return "quantize";
        case kStDequantize: return "dequantize";
        case kStSplit1Syn:
        case kStSplit1SynQ: return "dfb_split_synthesis";
        case kStSplit2Syn:
        case kStSplit2SynQ: return "dfb_split2_synthesis";
        case kStLevelSyn:
        case kStLevelSynQ: return "dfb12_lp_synthesis";
        default: return "unknown";
    }
}

hipError_t launch_stage_raw(const StageDesc& d, hipStream_t st) {
    switch (d.type) {
        case kStLevelAna:
        case kStLevelAnaQ: return launch_level_analysis(d.u.la, d.lo_r, st);
        case kStLevelSyn:
        case kStLevelSynQ: return launch_level_synthesis(d.u.ls, d.lo_r, st);
        case kStSplit1Ana:
        case kStSplit1AnaQ: return launch_dfb_split_analysis(d.u.sp, d.lift, d.batch, st);
        case kStSplit2Ana:
        case kStSplit2AnaQ: return launch_dfb_split2_analysis(d.u.sp, d.lift, d.batch, st);
        case kStSplit1Syn:
        case kStSplit1SynQ: return launch_dfb_split_synthesis(d.u.sp, d.lift, d.batch, st);
        case kStSplit2Syn:
        case kStSplit2SynQ: return launch_dfb_split2_synthesis(d.u.sp, d.lift, d.batch, st);
        case kStSplit3Ana:
        case kStSplit3AnaQ: return launch_dfb_split3_analysis(d.u.sp, d.lift, d.batch, st);
        case kStSplit3Syn:
        case kStSplit3SynQ: return launch_dfb_split3_synthesis(d.u.sp, d.lift, d.batch, st);
        case kStPartial: return launch_lowpass_partial(d.u.q, d.batch, st);
        case kStQuantize: return launch_quantize(d.u.q, d.batch, st);
        case kStDequantize: return launch_dequantize(d.u.q, d.batch, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

namespace ct {

int launch_stage(const StageDesc& d, hipStream_t st) {
    CT_PROFILED_ALG(stage_name(d.type), d.bytes, d.alg, launch_stage_raw(d, st), st);
    return CT_OK;
}

int launch_chain(const std::vector<StageDesc>& chain, hipStream_t st) {
    for (const StageDesc& d : chain) {
        const int rc = launch_stage(d, st);
        if (rc != CT_OK) return rc;
    }
    return CT_OK;
}

namespace {

// A second stream per device, and a fork and a join event, for chains whose
// level-1 split passes run beside the coarser levels. Created at first use
// and kept until the process ends; default priority, non-blocking.
struct Side {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_side_mu;
Side g_side[64];

bool is_level_stage(const StageDesc& d) {
    return d.type == kStLevelAna || d.type == kStLevelAnaQ || d.type == kStLevelSyn || d.type == kStLevelSynQ;
}
bool is_split_stage(const StageDesc& d) {
    switch (d.type) {
        case kStSplit1Ana: case kStSplit2Ana: case kStSplit3Ana: case kStSplit1AnaQ: case kStSplit2AnaQ:
        case kStSplit3AnaQ: case kStSplit1Syn: case kStSplit2Syn: case kStSplit3Syn: case kStSplit1SynQ:
        case kStSplit2SynQ: case kStSplit3SynQ:
            return true;
        default:
            return false;
    }
}

}  // namespace

// The level-1 split passes of a transform chain (stages [a0, a1)) depend only
// on the level-1 LP stage of the analysis (stage 0), or on nothing in the
// synthesis, and nothing but the level-1 LP synthesis (stage a1) depends on
// them; the coarser levels use their own channel buffers. So they run on a
// second stream beside the rest of the chain: the device overlaps the long
// level-1 passes with the short, latency-bound coarse levels. The results
// are those of launch_chain (each stage computes the same operations).
int launch_chain_forked(const std::vector<StageDesc>& chain, hipStream_t st) {
    const char* serial = getenv("CT_SERIAL_LEVELS");
    if (serial && *serial == '1') return launch_chain(chain, st);
    // find the level-1 split passes: analysis, right after the first LP
    // stage; synthesis, right before the last one
    const size_t n = chain.size();
    size_t a0 = 0, a1 = 0;
    bool analysis = false;
    if (n > 2 && (chain[0].type == kStLevelAna || chain[0].type == kStLevelAnaQ)) {
        analysis = true;
        a0 = a1 = 1;
        while (a1 < n && is_split_stage(chain[a1])) ++a1;
        if (a1 == n || !is_level_stage(chain[a1])) return launch_chain(chain, st);   // a single level
    } else if (n > 2 && (chain[n - 1].type == kStLevelSyn || chain[n - 1].type == kStLevelSynQ)) {
        a1 = n - 1;
        a0 = a1;
        while (a0 > 0 && is_split_stage(chain[a0 - 1])) --a0;
        if (a0 == 0) return launch_chain(chain, st);                                  // a single level
    } else {
        return launch_chain(chain, st);
    }
    if (a0 == a1) return launch_chain(chain, st);                                     // no level-1 split
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return CT_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_side_mu);
    Side& side = g_side[dev];
    if (!side.s) {
        // all three or none
        Side n;
        if (hipStreamCreateWithFlags(&n.s, hipStreamNonBlocking) != hipSuccess) return CT_ERR_HIP;
        if (hipEventCreateWithFlags(&n.fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&n.join, hipEventDisableTiming) != hipSuccess) {
            if (n.fork) hipEventDestroy(n.fork);
            hipStreamDestroy(n.s);
            return CT_ERR_HIP;
        }
        side = n;
    }
    auto run = [&](size_t b, size_t e, hipStream_t s) -> int {
        for (size_t i = b; i < e; ++i) {
            const int rc = launch_stage(chain[i], s);
            if (rc != CT_OK) return rc;
        }
        return CT_OK;
    };
    // analysis: stage 0 on the caller's stream first; then the level-1
    // passes on the side stream and the coarser levels on the caller's.
    // synthesis: the level-1 passes on the side stream from the start, the
    // coarser levels on the caller's, both joined before the last LP stage.
    int rc = analysis ? run(0, 1, st) : CT_OK;
    if (rc != CT_OK) return rc;
    if (hipEventRecord(side.fork, st) != hipSuccess || hipStreamWaitEvent(side.s, side.fork, 0) != hipSuccess)
        return CT_ERR_HIP;
    rc = run(a0, a1, side.s);
    // the join is enqueued whatever happened, so that the caller's stream
    // never runs ahead of work left on the side stream
    const bool joined = hipEventRecord(side.join, side.s) == hipSuccess;
    if (rc == CT_OK) rc = analysis ? run(a1, n, st) : run(0, a0, st);
    if (!joined || hipStreamWaitEvent(st, side.join, 0) != hipSuccess) return CT_ERR_HIP;
    if (rc == CT_OK && !analysis) rc = run(a1, n, st);
    return rc;
}

}  // namespace ct

namespace {

int transform(const ct_geom* geom, int32_t batch, const float* in, float* out, void* ws,
              size_t ws_bytes, hipStream_t st, Mode mode) {
    Geometry g;
    int rc = check_common(geom, batch, &g);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!in || !out || !ws) return CT_ERR_ARG;
    const Workspace w = workspace_layout(g, batch);
    if (ws_bytes < w.total) return CT_ERR_WORKSPACE;
    if (!constants(g.filters).ok) return CT_ERR_UNSUPPORTED;
    if (fault_injected()) return CT_ERR_HIP;
    std::vector<StageDesc> chain;
    int tune[kMaxLevels];
    tuned_codes(g, batch, tune);
    build_transform_chain(g, batch, int(mode), in, out, static_cast<char*>(ws), w, tune, chain);
    rc = launch_chain_forked(chain, st);
    if (rc != CT_OK) return rc;
    if (mode == Mode::ForwardAdjoint) {
        const int64_t RC = int64_t(g.R) * g.C;
        float* D = reinterpret_cast<float*>(static_cast<char*>(ws) + w.d_off);
        CT_PROFILED("pad_fold", 4.0 * batch * (double(RC) + double(g.H) * g.W),
                    launch_pad_fold(CView{D, RC, g.C}, g.R, g.C,
                                    View{out, int64_t(g.H) * g.W, g.W}, g.H, g.W, batch, st),
                    st);
    }
    return CT_OK;
}

}  // namespace

namespace ct {

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int fill_quant_args(const Geometry& g, QuantArgs* a) {
    if (g.nsub + 1 > int(sizeof(a->sub_off) / sizeof(a->sub_off[0]))) return CT_ERR_GEOM;
    std::vector<ct_subband> table(g.nsub);
    subband_table(g, table.data(), g.nsub);
    for (int s = 0; s < g.nsub; ++s) a->sub_off[s] = int(table[s].offset);
    a->sub_off[g.nsub] = int(g.ncoef);
    a->nsub = g.nsub;
    a->ncoef = g.ncoef;
    a->nq = g.ncoef;
    a->in_plane = g.ncoef;
    a->low_n = g.low_n;
    int64_t parts = (g.low_n + 4095) / 4096;
    if (parts < 1) parts = 1;
    if (parts > kMaxPart) parts = kMaxPart;
    a->nparts = int(parts);
    return CT_OK;
}

// Quantiser stages: lowpass partials, then the indices.
int build_quant_chain(const Geometry& g, int batch, const float* coeffs, const float* steps,
                      int steps_stride, int16_t* idx, float* side, char* ws, const Workspace& w,
                      std::vector<StageDesc>& chain) {
    StageDesc d;
    memset(&d, 0, sizeof(d));
    int rc = fill_quant_args(g, &d.u.q);
    if (rc != CT_OK) return rc;
    QuantArgs& a = d.u.q;
    a.coeffs = coeffs;
    a.idx = idx;
    a.side = side;
    a.steps = steps;
    a.steps_stride = steps_stride;
    a.partials = reinterpret_cast<float*>(ws + w.part_off);
    a.vec8 = g.ncoef % 8 == 0 && aligned16(coeffs) && aligned16(idx);
    d.batch = batch;
    d.type = kStPartial;
    d.ntiles = a.nparts * batch;
    d.bytes = 4.0 * batch * double(g.low_n);
    d.alg = 0.0;                            // the lowpass is read again by the next pass
    chain.push_back(d);
    d.type = kStQuantize;
    d.ntiles = int((g.ncoef + 4095) / 4096) * batch;
    d.bytes = 6.0 * batch * double(g.ncoef);
    d.alg = d.bytes;
    chain.push_back(d);
    return CT_OK;
}

int build_lowpass_quant_chain(const Geometry& g, int batch, const float* low, int64_t low_plane,
                              const float* steps, int steps_stride, int16_t* idx, float* side,
                              char* ws, const Workspace& w, std::vector<StageDesc>& chain) {
    StageDesc d;
    memset(&d, 0, sizeof(d));
    int rc = fill_quant_args(g, &d.u.q);
    if (rc != CT_OK) return rc;
    QuantArgs& a = d.u.q;
    a.coeffs = low;
    a.in_plane = low_plane;
    a.nq = g.low_n;
    a.idx = idx;
    a.side = side;
    a.steps = steps;
    a.steps_stride = steps_stride;
    a.partials = reinterpret_cast<float*>(ws + w.part_off);
    a.vec8 = g.ncoef % 8 == 0 && low_plane % 8 == 0 && g.low_n % 8 == 0 && aligned16(low) && aligned16(idx);
    d.batch = batch;
    d.type = kStPartial;
    d.ntiles = a.nparts * batch;
    d.bytes = 4.0 * batch * double(g.low_n);
    d.alg = 0.0;
    chain.push_back(d);
    d.type = kStQuantize;
    d.ntiles = int((g.low_n + 4095) / 4096) * batch;
    d.bytes = 6.0 * batch * double(g.low_n);
    // the float lowpass is the caller's output only when it sits in coeffs
    d.alg = (low_plane == g.ncoef ? 6.0 : 2.0) * batch * double(g.low_n);
    chain.push_back(d);
    return CT_OK;
}

int build_dequant_chain(const Geometry& g, int batch, const int16_t* idx, const float* steps,
                        int steps_stride, const float* side, float* coeffs,
                        std::vector<StageDesc>& chain) {
    StageDesc d;
    memset(&d, 0, sizeof(d));
    int rc = fill_quant_args(g, &d.u.q);
    if (rc != CT_OK) return rc;
    QuantArgs& a = d.u.q;
    a.idx_in = idx;
    a.coeffs_out = coeffs;
    a.vec8 = g.ncoef % 8 == 0 && aligned16(idx) && aligned16(coeffs);
    a.side = const_cast<float*>(side);
    a.steps = steps;
    a.steps_stride = steps_stride;
    d.batch = batch;
    d.type = kStDequantize;
    d.ntiles = int((g.ncoef + 4095) / 4096) * batch;
    d.bytes = 6.0 * batch * double(g.ncoef);
    d.alg = d.bytes;
    chain.push_back(d);
    return CT_OK;
}

}  // namespace ct

extern "C" {

int ct_layout_query(const ct_geom* geom, ct_layout* out, ct_subband* table, int32_t cap) {
    if (!geom || !out) return CT_ERR_ARG;
    if (cap < 0 || (cap > 0 && !table)) return CT_ERR_ARG;
    Geometry g;
    int rc = resolve(geom, &g);
    if (rc != CT_OK) return rc;
    out->pad_h = g.R;
    out->pad_w = g.C;
    out->exp2 = g.e;
    out->nsub = g.nsub;
    out->ncoef = g.ncoef;
    if (cap > 0) subband_table(g, table, cap);
    return CT_OK;
}

int ct_workspace_bytes(const ct_geom* geom, int32_t batch, size_t* bytes) {
    if (bytes) *bytes = 0;
    if (!bytes) return CT_ERR_ARG;
    Geometry g;
    int rc = check_common(geom, batch, &g);
    if (rc != CT_OK) return rc;
    *bytes = workspace_layout(g, batch).total;
    return CT_OK;
}

int ct_forward(const ct_geom* geom, int32_t batch, const float* planes, float* coeffs, void* ws,
               size_t ws_bytes, hipStream_t stream) {
    return transform(geom, batch, planes, coeffs, ws, ws_bytes, stream, Mode::Forward);
}

int ct_inverse(const ct_geom* geom, int32_t batch, const float* coeffs, float* planes, void* ws,
               size_t ws_bytes, hipStream_t stream) {
    return transform(geom, batch, coeffs, planes, ws, ws_bytes, stream, Mode::Inverse);
}

int ct_forward_adjoint(const ct_geom* geom, int32_t batch, const float* gcoeffs, float* gplanes,
                       void* ws, size_t ws_bytes, hipStream_t stream) {
    return transform(geom, batch, gcoeffs, gplanes, ws, ws_bytes, stream, Mode::ForwardAdjoint);
}

int ct_inverse_adjoint(const ct_geom* geom, int32_t batch, const float* gplanes, float* gcoeffs,
                       void* ws, size_t ws_bytes, hipStream_t stream) {
    return transform(geom, batch, gplanes, gcoeffs, ws, ws_bytes, stream, Mode::InverseAdjoint);
}

int ct_quantize(const ct_geom* geom, int32_t batch, const float* coeffs, const float* steps,
                int32_t steps_stride, int16_t* idx, float* side, void* ws, size_t ws_bytes,
                hipStream_t stream) {
    Geometry g;
    int rc = check_common(geom, batch, &g);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!coeffs || !steps || !idx || !side || !ws) return CT_ERR_ARG;
    if (steps_stride < 0 || (steps_stride > 0 && steps_stride < g.nsub)) return CT_ERR_ARG;
    const Workspace w = workspace_layout(g, batch);
    if (ws_bytes < w.total) return CT_ERR_WORKSPACE;
    if (fault_injected()) return CT_ERR_HIP;
    std::vector<StageDesc> chain;
    rc = build_quant_chain(g, batch, coeffs, steps, steps_stride, idx, side,
                           static_cast<char*>(ws), w, chain);
    if (rc != CT_OK) return rc;
    return launch_chain(chain, stream);
}

}  // extern "C"

namespace ct {

// Argument checks of ct_quantize (host only).
int check_quantize(const ct_geom* geom, int32_t batch, const float* coeffs, const float* steps,
                   int32_t steps_stride, const int16_t* idx, const float* side) {
    Geometry g;
    const int rc = check_common(geom, batch, &g);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!coeffs || !steps || !idx || !side) return CT_ERR_ARG;
    if (steps_stride < 0 || (steps_stride > 0 && steps_stride < g.nsub)) return CT_ERR_ARG;
    return CT_OK;
}

// ct_quantize with the lowpass partials at `partials` (device memory of
// `partial_bytes` bytes) instead of in a caller workspace.
int quantize_with_partials(const ct_geom* geom, int32_t batch, const float* coeffs,
                           const float* steps, int32_t steps_stride, int16_t* idx, float* side,
                           void* partials, size_t partial_bytes, hipStream_t stream) {
    int rc = check_quantize(geom, batch, coeffs, steps, steps_stride, idx, side);
    if (rc != CT_OK || batch == 0) return rc;
    Geometry g;
    rc = check_common(geom, batch, &g);
    if (rc != CT_OK) return rc;
    if (!partials) return CT_ERR_ARG;
    if (partial_bytes < quantize_partial_bytes(batch)) return CT_ERR_WORKSPACE;
    if (fault_injected()) return CT_ERR_HIP;
    Workspace w;                   // only the partials are used, at offset 0
    w.part_off = 0;
    std::vector<StageDesc> chain;
    rc = build_quant_chain(g, batch, coeffs, steps, steps_stride, idx, side,
                           static_cast<char*>(partials), w, chain);
    if (rc != CT_OK) return rc;
    return launch_chain(chain, stream);
}

}  // namespace ct

extern "C" {

int ct_dequantize(const ct_geom* geom, int32_t batch, const int16_t* idx, const float* steps,
                  int32_t steps_stride, const float* side, float* coeffs, hipStream_t stream) {
    Geometry g;
    int rc = check_common(geom, batch, &g);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!coeffs || !steps || !idx || !side) return CT_ERR_ARG;
    if (steps_stride < 0 || (steps_stride > 0 && steps_stride < g.nsub)) return CT_ERR_ARG;
    if (fault_injected()) return CT_ERR_HIP;
    std::vector<StageDesc> chain;
    rc = build_dequant_chain(g, batch, idx, steps, steps_stride, side, coeffs, chain);
    if (rc != CT_OK) return rc;
    return launch_chain(chain, stream);
}

int ct_encode(const ct_geom* geom, int32_t batch, const float* planes, const float* steps,
              int32_t steps_stride, int16_t* idx, float* side, float* coeffs, void* ws,
              size_t ws_bytes, hipStream_t stream) {
    Geometry g;
    int rc = check_common(geom, batch, &g);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!planes || !steps || !idx || !side || !ws) return CT_ERR_ARG;
    if (steps_stride < 0 || (steps_stride > 0 && steps_stride < g.nsub)) return CT_ERR_ARG;
    const Workspace w = workspace_layout(g, batch);
    if (ws_bytes < w.total) return CT_ERR_WORKSPACE;
    if (!constants(g.filters).ok) return CT_ERR_UNSUPPORTED;
    if (fault_injected()) return CT_ERR_HIP;
    char* wsc = static_cast<char*>(ws);
    const FusedQuant fq{idx, steps, steps_stride, nullptr};
    std::vector<StageDesc> chain;
    int tune[kMaxLevels];
    tuned_codes(g, batch, tune);
    build_transform_chain(g, batch, kModeForward, planes, coeffs, wsc, w, tune, chain, &fq);
    const float* low = coeffs ? coeffs : reinterpret_cast<const float*>(wsc + w.low_off);
    rc = build_lowpass_quant_chain(g, batch, low, coeffs ? g.ncoef : g.low_n, steps, steps_stride, idx,
                                   side, wsc, w, chain);
    if (rc != CT_OK) return rc;
    return launch_chain_forked(chain, stream);
}

int ct_encode_rgb(const ct_geom* geom, int32_t frames, const uint8_t* rgb, const float* steps,
                  int32_t steps_stride, int16_t* idx, float* side, void* ws, size_t ws_bytes,
                  hipStream_t stream) {
    if (frames < 0 || frames > 65535 / 3) return CT_ERR_ARG;
    const int32_t batch = 3 * frames;
    Geometry g;
    int rc = check_common(geom, batch, &g);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!rgb || !steps || !idx || !side || !ws) return CT_ERR_ARG;
    if (steps_stride < 0 || (steps_stride > 0 && steps_stride < g.nsub)) return CT_ERR_ARG;
    if (int64_t(frames) * g.H * g.W * 3 >= (int64_t(1) << 40)) return CT_ERR_ARG;
    const Workspace w = workspace_layout(g, batch);
    if (ws_bytes < w.total) return CT_ERR_WORKSPACE;
    if (!constants(g.filters).ok) return CT_ERR_UNSUPPORTED;
    if (fault_injected()) return CT_ERR_HIP;
    char* wsc = static_cast<char*>(ws);
    const FusedQuant fq{idx, steps, steps_stride, nullptr};
    std::vector<StageDesc> chain;
    int tune[kMaxLevels];
    tuned_codes(g, batch, tune);
    build_transform_chain(g, batch, kModeForward, nullptr, nullptr, wsc, w, tune, chain, &fq, rgb);
    rc = build_lowpass_quant_chain(g, batch, reinterpret_cast<const float*>(wsc + w.low_off), g.low_n, steps,
                                   steps_stride, idx, side, wsc, w, chain);
    if (rc != CT_OK) return rc;
    return launch_chain_forked(chain, stream);
}

int ct_decode(const ct_geom* geom, int32_t batch, const int16_t* idx, const float* steps,
              int32_t steps_stride, const float* side, float* planes, void* ws, size_t ws_bytes,
              hipStream_t stream) {
    Geometry g;
    int rc = check_common(geom, batch, &g);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!idx || !steps || !side || !planes || !ws) return CT_ERR_ARG;
    if (steps_stride < 0 || (steps_stride > 0 && steps_stride < g.nsub)) return CT_ERR_ARG;
    const Workspace w = workspace_layout(g, batch);
    if (ws_bytes < w.total) return CT_ERR_WORKSPACE;
    if (!constants(g.filters).ok) return CT_ERR_UNSUPPORTED;
    if (fault_injected()) return CT_ERR_HIP;
    const FusedQuant fq{const_cast<int16_t*>(idx), steps, steps_stride, side};
    std::vector<StageDesc> chain;
    int tune[kMaxLevels];
    tuned_codes(g, batch, tune);
    build_transform_chain(g, batch, kModeInverse, nullptr, planes, static_cast<char*>(ws), w, tune, chain, &fq);
    return launch_chain_forked(chain, stream);
}

int ct_profile_enable(int32_t on, int32_t max_launches) {
    Profiler& p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    if (on) {
        if (max_launches <= 0) max_launches = 16384;
        if (p.pool.size() < size_t(2) * max_launches) {
            while (p.pool.size() < size_t(2) * max_launches) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return CT_ERR_HIP;
                p.pool.push_back(e);
            }
        }
        p.on = true;
        return CT_OK;
    }
    p.on = false;
    for (const ProfRecord& r : p.recs) hipEventSynchronize(r.b);
    for (hipEvent_t e : p.pool) hipEventDestroy(e);
    p.pool.clear();
    p.recs.clear();
    p.next = 0;
    p.dropped = false;
    return CT_OK;
}

int ct_profile_collect(ct_kernel_stat* out, int32_t cap, int32_t* n) {
    if (!n || cap < 0 || (cap > 0 && !out)) return CT_ERR_ARG;
    Profiler& p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    std::vector<std::string> order;
    std::map<std::string, ct_kernel_stat> agg;
    int rc = CT_OK;
    for (const ProfRecord& r : p.recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            rc = CT_ERR_HIP;
            continue;
        }
        auto it = agg.find(r.name);
        if (it == agg.end()) {
            ct_kernel_stat z;
            memset(&z, 0, sizeof(z));
            strncpy(z.name, r.name, sizeof(z.name) - 1);
            it = agg.emplace(r.name, z).first;
            order.push_back(r.name);
        }
        it->second.launches += 1;
        it->second.total_ms += ms;
        it->second.bytes += r.bytes;
        it->second.alg_bytes += r.alg;
    }
    *n = int32_t(order.size());
    for (int32_t i = 0; i < cap && i < int32_t(order.size()); ++i) out[i] = agg[order[i]];
    if (p.dropped && rc == CT_OK) rc = CT_ERR_UNSUPPORTED;
    p.recs.clear();
    p.next = 0;
    p.dropped = false;
    return rc;
}

const char* ct_strerror(int code) {
    switch (code) {
        case CT_OK: return "success";
        case CT_ERR_ARG: return "invalid argument";
        case CT_ERR_GEOM: return "unsupported geometry";
        case CT_ERR_WORKSPACE: return "workspace too small";
        case CT_ERR_HIP: return "HIP runtime error";
        case CT_ERR_UNSUPPORTED: return "unsupported request";
        default: return "unknown error";
    }
}

}  // extern "C"

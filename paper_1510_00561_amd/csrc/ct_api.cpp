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

#include "ct_internal.h"
#include "ct_kernels.h"

using namespace ct;

namespace {

enum class Mode { Forward, Inverse, ForwardAdjoint, InverseAdjoint };

Taps5 taps_h() {
    const Constants& k = constants();
    Taps5 t;
    for (int i = 0; i < 5; ++i) t.t[i] = float(k.hbar[i]);
    return t;
}

Taps5 taps_g() {
    const Constants& k = constants();
    Taps5 t;
    for (int i = 0; i < 4; ++i) t.t[i] = float(k.gbar[i]);
    t.t[4] = 0.f;
    return t;
}

Lift lift_for(Mode m) {
    const Constants& k = constants();
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
void scale_table(int l, int sign, float* out) {
    int e[kMaxDirs];
    dfb_scale_exponents(l, e);
    const double z = constants().zeta;
    for (int k = 0; k < (1 << l); ++k) out[k] = float(pow(z, double(sign * e[k])));
}

bool fault_injected() {
    const char* f = getenv("CT_FAULT_INJECT");
    return f && strcmp(f, "launch") == 0;
}

// ------------------------------------------------------------ profiling
// Event pairs around launches, recorded only while enabled. The pool is
// created by ct_profile_enable so that recording never allocates.
struct ProfRecord {
    const char* name;
    double bytes;
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
Profiler& profiler() {
    static Profiler p;
    return p;
}

struct ProfScope {
    const char* name;
    double bytes;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(const char* n, double by, hipStream_t s) : name(n), bytes(by), st(s) {
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
    void done() {
        if (!a) return;
        Profiler& p = profiler();
        std::lock_guard<std::mutex> lock(p.mu);
        hipEventRecord(b, st);
        p.recs.push_back(ProfRecord{name, bytes, a, b});
    }
};

#define CT_LAUNCH(name, bytes, expr)                      \
    do {                                                  \
        ProfScope ct_prof_scope_(name, double(bytes), st); \
        if ((expr) != hipSuccess) return CT_ERR_HIP;      \
        ct_prof_scope_.done();                            \
    } while (0)

int check_common(const ct_geom* geom, int32_t batch, Geometry* g) {
    if (!geom) return CT_ERR_ARG;
    if (batch < 0 || batch > 65535) return CT_ERR_ARG;
    return resolve(geom, g);
}

// Groups of DFB tree levels >= 3 run per pass: pairs from the top, then a
// single trailing level when their count is odd.
int split_groups(int l, int* first, int* count) {
    int n = 0;
    for (int t = 3; t <= l; t += 2) {
        first[n] = t;
        count[n] = (t + 1 <= l) ? 2 : 1;
        ++n;
    }
    return n;
}

// Analysis direction: image -> coefficients (forward, inverse adjoint).
int run_analysis(const Geometry& g, int batch, const float* planes, float* coeffs, char* ws,
                 const Workspace& w, Mode mode, hipStream_t st) {
    const bool fwd = mode == Mode::Forward;
    const Taps5 lo = fwd ? taps_h() : taps_g();
    const Taps5 up = fwd ? taps_g() : taps_h();
    const int lo_r = fwd ? 4 : 3, up_r = fwd ? 3 : 4;
    const Lift L = lift_for(mode);
    const int64_t RC = int64_t(g.R) * g.C;
    float* A = reinterpret_cast<float*>(ws + w.a_off);
    float* Bf = reinterpret_cast<float*>(ws + w.b_off);
    for (int j = 1; j <= g.J; ++j) {
        const int Rj = g.R >> (j - 1), Cj = g.C >> (j - 1);
        CView src;
        int src_h = Rj, src_w = Cj, pad = kPadNone;
        if (j == 1) {
            src = CView{planes, int64_t(g.H) * g.W, g.W};
            src_h = g.H;
            src_w = g.W;
            pad = fwd ? kPadReflect : kPadZero;
        } else {
            src = CView{reinterpret_cast<const float*>(ws + w.c_off[j - 1]), int64_t(Rj) * Cj, Cj};
        }
        View c_out = (j == g.J)
                         ? View{coeffs, g.ncoef, Cj / 2}
                         : View{reinterpret_cast<float*>(ws + w.c_off[j]), int64_t(Rj / 2) * (Cj / 2), Cj / 2};
        const int l = g.l[j - 1];
        float* level = coeffs + g.level_off[j];
        const int64_t q4 = int64_t(Rj) * Cj / 4;
        float sc[kMaxDirs];
        scale_table(l, fwd ? +1 : -1, sc);
        Quad quad;
        if (l == 2) {
            for (int k = 0; k < 4; ++k) {
                quad.p[k] = level + k * q4;
                quad.scale[k] = sc[k];
            }
            quad.plane = g.ncoef;
        } else {
            for (int k = 0; k < 4; ++k) {
                quad.p[k] = A + k * q4;
                quad.scale[k] = 1.f;
            }
            quad.plane = RC;
        }
        const double lvl_bytes = 8.0 * batch * double(Rj) * Cj;
        const double lp_bytes = 4.0 * batch *
            (double(src_h) * src_w + double(Rj / 2) * (Cj / 2) + double(Rj) * Cj);
        CT_LAUNCH("lp_dfb12_analysis", lp_bytes,
                  launch_lp_dfb12_analysis(src, src_h, src_w, pad, Rj, Cj, c_out, quad, lo, lo_r,
                                           up, up_r, L, batch, st));
        int first[4], count[4];
        const int ng = split_groups(l, first, count);
        float* cur = A;
        float* other = Bf;
        for (int gi = 0; gi < ng; ++gi) {
            const bool last = gi == ng - 1;
            SplitArgs a;
            memset(&a, 0, sizeof(a));
            a.t = first[gi];
            a.Rj = Rj;
            a.Cj = Cj;
            a.parent = cur;
            a.parent_plane = RC;
            a.plane_elems = int64_t(Rj) * Cj;
            if (last) {
                a.child = level;
                a.child_plane = g.ncoef;
                a.use_scale = 1;
                memcpy(a.scale, sc, sizeof(float) * (1 << l));
            } else {
                a.child = other;
                a.child_plane = RC;
            }
            if (count[gi] == 2)
                CT_LAUNCH("dfb_split2_analysis", lvl_bytes, launch_dfb_split2_analysis(a, L, batch, st));
            else
                CT_LAUNCH("dfb_split_analysis", lvl_bytes, launch_dfb_split_analysis(a, L, batch, st));
            float* tmp = cur;
            cur = other;
            other = tmp;
        }
    }
    return CT_OK;
}

// Synthesis direction: coefficients -> image (inverse, forward adjoint).
int run_synthesis(const Geometry& g, int batch, const float* coeffs, float* planes, char* ws,
                  const Workspace& w, Mode mode, hipStream_t st) {
    const bool inv = mode == Mode::Inverse;
    const Taps5 lo = inv ? taps_h() : taps_g();
    const Taps5 up = inv ? taps_g() : taps_h();
    const int lo_r = inv ? 4 : 3, up_r = inv ? 3 : 4;
    const Lift L = lift_for(mode);
    const int64_t RC = int64_t(g.R) * g.C;
    float* D = reinterpret_cast<float*>(ws + w.d_off);
    float* A = reinterpret_cast<float*>(ws + w.a_off);
    float* Bf = reinterpret_cast<float*>(ws + w.b_off);
    for (int j = g.J; j >= 1; --j) {
        const int Rj = g.R >> (j - 1), Cj = g.C >> (j - 1);
        const int l = g.l[j - 1];
        const float* level = coeffs + g.level_off[j];
        const int64_t q4 = int64_t(Rj) * Cj / 4;
        const double lvl_bytes = 8.0 * batch * double(Rj) * Cj;
        float sc[kMaxDirs];
        scale_table(l, inv ? -1 : +1, sc);
        Quad quad;
        if (l == 2) {
            for (int k = 0; k < 4; ++k) {
                quad.p[k] = const_cast<float*>(level) + k * q4;
                quad.scale[k] = sc[k];
            }
            quad.plane = g.ncoef;
        } else {
            int first[4], count[4];
            const int ng = split_groups(l, first, count);
            float* cur = A;
            float* other = Bf;
            for (int gi = ng - 1; gi >= 0; --gi) {
                SplitArgs a;
                memset(&a, 0, sizeof(a));
                a.t = first[gi];
                a.Rj = Rj;
                a.Cj = Cj;
                a.plane_elems = int64_t(Rj) * Cj;
                a.child = cur;            // output: the parents
                a.child_plane = RC;
                if (gi == ng - 1) {
                    a.parent = level;     // input: the final subbands
                    a.parent_plane = g.ncoef;
                    a.use_scale = 1;
                    memcpy(a.scale, sc, sizeof(float) * (1 << l));
                } else {
                    a.parent = other;
                    a.parent_plane = RC;
                }
                if (count[gi] == 2)
                    CT_LAUNCH("dfb_split2_synthesis", lvl_bytes,
                              launch_dfb_split2_synthesis(a, L, batch, st));
                else
                    CT_LAUNCH("dfb_split_synthesis", lvl_bytes,
                              launch_dfb_split_synthesis(a, L, batch, st));
                float* tmp = cur;
                cur = other;
                other = tmp;
            }
            // the last pass wrote into `other` (after the swap)
            for (int k = 0; k < 4; ++k) {
                quad.p[k] = other + k * q4;
                quad.scale[k] = 1.f;
            }
            quad.plane = RC;
        }
        CView c_in = (j == g.J)
                         ? CView{coeffs, g.ncoef, Cj / 2}
                         : CView{reinterpret_cast<const float*>(ws + w.c_off[j]), int64_t(Rj / 2) * (Cj / 2), Cj / 2};
        View x_out;
        int out_h = Rj, out_w = Cj;
        if (j == 1 && inv) {
            x_out = View{planes, int64_t(g.H) * g.W, g.W};
            out_h = g.H;
            out_w = g.W;
        } else if (j == 1) {
            x_out = View{D, RC, g.C};
        } else {
            x_out = View{reinterpret_cast<float*>(ws + w.c_off[j - 1]), int64_t(Rj) * Cj, Cj};
        }
        const double lps_bytes = 4.0 * batch *
            (double(Rj / 2) * (Cj / 2) + double(Rj) * Cj + double(out_h) * out_w);
        CT_LAUNCH("dfb12_lp_synthesis", lps_bytes,
                  launch_dfb12_lp_synthesis(quad, c_in, Rj, Cj, x_out, out_h, out_w, lo, lo_r, up,
                                            up_r, L, batch, st));
    }
    if (!inv) {
        CT_LAUNCH("pad_fold", 4.0 * batch * (double(RC) + double(g.H) * g.W),
                  launch_pad_fold(CView{D, RC, g.C}, g.R, g.C,
                                  View{planes, int64_t(g.H) * g.W, g.W}, g.H, g.W, batch, st));
    }
    return CT_OK;
}

int transform(const ct_geom* geom, int32_t batch, const float* in, float* out, void* ws,
              size_t ws_bytes, hipStream_t st, Mode mode) {
    Geometry g;
    int rc = check_common(geom, batch, &g);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!in || !out || !ws) return CT_ERR_ARG;
    const Workspace w = workspace_layout(g, batch);
    if (ws_bytes < w.total) return CT_ERR_WORKSPACE;
    if (!constants().ok) return CT_ERR_UNSUPPORTED;
    if (fault_injected()) return CT_ERR_HIP;
    char* wsb = static_cast<char*>(ws);
    if (mode == Mode::Forward || mode == Mode::InverseAdjoint)
        return run_analysis(g, batch, in, out, wsb, w, mode, st);
    return run_synthesis(g, batch, in, out, wsb, w, mode, st);
}

int fill_quant_args(const Geometry& g, QuantArgs* a) {
    if (g.nsub + 1 > int(sizeof(a->sub_off) / sizeof(a->sub_off[0]))) return CT_ERR_GEOM;
    ct_subband table[400];
    subband_table(g, table, 400);
    for (int s = 0; s < g.nsub; ++s) a->sub_off[s] = int(table[s].offset);
    a->sub_off[g.nsub] = int(g.ncoef);
    a->nsub = g.nsub;
    a->ncoef = g.ncoef;
    a->low_n = g.low_n;
    int64_t parts = (g.low_n + 4095) / 4096;
    if (parts < 1) parts = 1;
    if (parts > kMaxPart) parts = kMaxPart;
    a->nparts = int(parts);
    return CT_OK;
}

}  // namespace

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
    QuantArgs a;
    memset(&a, 0, sizeof(a));
    rc = fill_quant_args(g, &a);
    if (rc != CT_OK) return rc;
    a.coeffs = coeffs;
    a.idx = idx;
    a.side = side;
    a.steps = steps;
    a.steps_stride = steps_stride;
    a.partials = reinterpret_cast<float*>(static_cast<char*>(ws) + w.part_off);
    hipStream_t st = stream;
    CT_LAUNCH("lowpass_partial", 4.0 * batch * double(g.low_n), launch_lowpass_partial(a, batch, st));
    CT_LAUNCH("quantize", 6.0 * batch * double(g.ncoef), launch_quantize(a, batch, st));
    return CT_OK;
}

int ct_dequantize(const ct_geom* geom, int32_t batch, const int16_t* idx, const float* steps,
                  int32_t steps_stride, const float* side, float* coeffs, hipStream_t stream) {
    Geometry g;
    int rc = check_common(geom, batch, &g);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!coeffs || !steps || !idx || !side) return CT_ERR_ARG;
    if (steps_stride < 0 || (steps_stride > 0 && steps_stride < g.nsub)) return CT_ERR_ARG;
    if (fault_injected()) return CT_ERR_HIP;
    QuantArgs a;
    memset(&a, 0, sizeof(a));
    rc = fill_quant_args(g, &a);
    if (rc != CT_OK) return rc;
    a.idx_in = idx;
    a.coeffs_out = coeffs;
    a.side = const_cast<float*>(side);
    a.steps = steps;
    a.steps_stride = steps_stride;
    hipStream_t st = stream;
    CT_LAUNCH("dequantize", 6.0 * batch * double(g.ncoef), launch_dequantize(a, batch, st));
    return CT_OK;
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

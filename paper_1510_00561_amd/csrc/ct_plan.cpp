// Batched plans: many streams of uneven resolution and LP depth in one graph
// launch (host side).
//
// A plan owns a workspace slice per stream, the stage-descriptor table of
// every stream's chain (forward CT, quantise, dequantise, inverse CT) laid
// out group by group, and, with CT_PLAN_GRAPH, an instantiated HIP graph of
// the group launches. A group is the set of stages of one type at one chain
// position over all streams; its launch covers all their tiles.
//
// Autotuning (CT_PLAN_AUTOTUNE) picks, for every distinct LP level shape
// with three or more DFB tree levels, how many of the deeper tree levels run
// per streaming pass (one, two or three: halo 4, 12 or 28 rows) and the
// row-block height of those passes (the host's default, about half of it or
// about twice it), by timing every combination with HIP events. All choices
// compute the same float32 operations in the same order, so none changes a
// result. Choices are cached in a JSON file keyed by device architecture and
// shape (CT_AUTOTUNE_CACHE, default $HOME/.cache/ct_autotune.json).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "ct_batched.h"
#include "ct_internal.h"
#include "ct_kernels.h"
#include "ct_plan_internal.h"

using namespace ct;

struct ct_plan {
    int device = 0;
    std::vector<ct_stream_desc> streams;
    std::vector<Geometry> geoms;
    std::vector<Workspace> wls;
    std::vector<size_t> ws_off;
    char* ws = nullptr;
    std::vector<std::vector<StageDesc>> chains;     // per stream, chain order
    std::vector<int> grouping;                      // tune codes [stream * kMaxLevels + j]
    struct Group {
        int type, stage0, n, tiles;    // stages [stage0, stage0 + n) of d_stages / d_first
    };
    std::vector<Group> groups;
    StageDesc* d_stages = nullptr;
    int* d_first = nullptr;
    int nstages = 0;
    int total_items = 0;
    double bytes = 0, alg = 0;
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int autotuned = 0;
};

namespace {

// ---------------------------------------------------------------- autotune cache
std::string cache_path() {
    const char* p = getenv("CT_AUTOTUNE_CACHE");
    if (p && *p) return p;
    const char* home = getenv("HOME");
    return std::string(home ? home : ".") + "/.cache/ct_autotune.json";
}

// The cache is a flat JSON object {"key": integer, ...}.
std::map<std::string, int> load_cache() {
    std::map<std::string, int> m;
    FILE* f = fopen(cache_path().c_str(), "r");
    if (!f) return m;
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
    fclose(f);
    size_t i = 0;
    while ((i = text.find('"', i)) != std::string::npos) {
        const size_t j = text.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = text.substr(i + 1, j - i - 1);
        const size_t colon = text.find(':', j);
        if (colon == std::string::npos) break;
        m[key] = atoi(text.c_str() + colon + 1);
        i = text.find_first_of(",}", colon);
        if (i == std::string::npos) break;
    }
    return m;
}

void save_cache(const std::map<std::string, int>& m) {
    const std::string path = cache_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) mkdir(path.substr(0, slash).c_str(), 0755);   // may exist
    FILE* f = fopen(path.c_str(), "w");
    if (!f) return;   // no writable cache: the choices stay in this plan only
    fprintf(f, "{\n");
    size_t k = 0;
    for (const auto& kv : m) fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++k < m.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
}

std::string arch_name(int dev) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    return p.gcnArchName;
}

// Time the DFB split passes (analysis then synthesis) of one LP level shape
// with the given grouping and block height, using workspace buffers as
// scratch.
float time_level_splits(int Rj, int Cj, int l, int batch, int grouping, int height, float* A, float* B,
                        float* D, int64_t plane, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    int first[4], count[4], ng = 0;
    for (int t = 3; t <= l;) {
        const int c = t + grouping - 1 <= l ? grouping : l - t + 1;
        first[ng] = t;
        count[ng] = c;
        ++ng;
        t += c;
    }
    static hipError_t (*const ana[3])(const SplitArgs&, Lift, int, hipStream_t) = {
        launch_dfb_split_analysis, launch_dfb_split2_analysis, launch_dfb_split3_analysis};
    static hipError_t (*const syn[3])(const SplitArgs&, Lift, int, hipStream_t) = {
        launch_dfb_split_synthesis, launch_dfb_split2_synthesis, launch_dfb_split3_synthesis};
    Lift L{{-1.5f, -0.05f, 0.88f, 0.44f}, 1};
    auto run = [&]() -> bool {
        float* cur = A;
        float* other = B;
        for (int gi = 0; gi < ng; ++gi) {
            SplitArgs a;
            memset(&a, 0, sizeof(a));
            a.t = first[gi];
            a.Rj = Rj;
            a.Cj = Cj;
            a.parent = cur;
            a.parent_plane = plane;
            a.child = gi == ng - 1 ? D : other;
            a.child_plane = plane;
            a.plane_elems = int64_t(Rj) * Cj;
            a.bh = split_block_rows(a, batch, count[gi], height);
            hipError_t e = ana[count[gi] - 1](a, L, batch, st);
            if (e != hipSuccess) return false;
            std::swap(cur, other);
        }
        float* cur2 = A;
        float* other2 = B;
        for (int gi = ng - 1; gi >= 0; --gi) {
            SplitArgs a;
            memset(&a, 0, sizeof(a));
            a.t = first[gi];
            a.Rj = Rj;
            a.Cj = Cj;
            a.parent = gi == ng - 1 ? D : other2;
            a.parent_plane = plane;
            a.child = cur2;
            a.child_plane = plane;
            a.plane_elems = int64_t(Rj) * Cj;
            a.bh = split_block_rows(a, batch, count[gi], height);
            hipError_t e = syn[count[gi] - 1](a, L, batch, st);
            if (e != hipSuccess) return false;
            std::swap(cur2, other2);
        }
        return true;
    };
    if (!run()) return -1.f;
    if (hipEventRecord(e0, st) != hipSuccess) return -1.f;
    for (int r = 0; r < 3; ++r)
        if (!run()) return -1.f;
    if (hipEventRecord(e1, st) != hipSuccess) return -1.f;
    if (hipEventSynchronize(e1) != hipSuccess) return -1.f;
    float ms = 0;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.f;
    return ms;
}

// A cached code the chain builder can use (anything else is tuned again).
bool valid_tune(int code) {
    const int g = tune_grouping(code), h = tune_height(code);
    return code >= 0 && (code >> 6) == 0 && g >= 1 && g <= 3 && h <= kHeightTall;
}

int autotune(ct_plan* p, hipStream_t st) {
    std::map<std::string, int> cache = load_cache();
    const std::string arch = arch_name(p->device);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return CT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return CT_ERR_HIP;
    }
    bool dirty = false;
    int rc = CT_OK;
    for (size_t s = 0; s < p->streams.size() && rc == CT_OK; ++s) {
        const Geometry& g = p->geoms[s];
        const int batch = p->streams[s].batch;
        char* ws = p->ws + p->ws_off[s];
        const Workspace& w = p->wls[s];
        for (int j = 1; j <= g.J; ++j) {
            const int l = g.l[j - 1];
            if (l < 3) continue;    // no split pass
            const int Rj = g.R >> (j - 1), Cj = g.C >> (j - 1);
            char key[160];
            snprintf(key, sizeof(key), "%s|split_tune|%dx%d|l%d|b%d", arch.c_str(), Rj, Cj, l, batch);
            auto it = cache.find(key);
            int choice;
            if (it != cache.end() && valid_tune(it->second)) {
                choice = it->second;
            } else {
                float* A = reinterpret_cast<float*>(ws + w.a_off);
                float* B = reinterpret_cast<float*>(ws + w.b_off);
                float* D = reinterpret_cast<float*>(ws + w.d_off);
                const int64_t plane = int64_t(g.R) * g.C;
                // every grouping that differs for this depth (up to l - 2
                // levels per pass), at each of the three block heights
                float best = -1.f;
                choice = tune_code(1, kHeightDefault);
                for (int grp = 1; grp <= 3 && grp <= l - 2 && rc == CT_OK; ++grp)
                    for (int hm = kHeightDefault; hm <= kHeightTall; ++hm) {
                        const float ms = time_level_splits(Rj, Cj, l, batch, grp, hm, A, B, D, plane, st, e0, e1);
                        if (ms < 0) {
                            rc = CT_ERR_HIP;
                            break;
                        }
                        if (best < 0 || ms < best) {
                            best = ms;
                            choice = tune_code(grp, hm);
                        }
                    }
                if (rc != CT_OK) break;
                cache[key] = choice;
                dirty = true;
            }
            p->grouping[s * kMaxLevels + (j - 1)] = choice;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (dirty) save_cache(cache);
    p->autotuned = 1;
    return rc;
}

// The group launches of a plan, in chain order.
hipError_t launch_groups(const ct_plan* p, hipStream_t st) {
    for (const ct_plan::Group& g : p->groups) {
        const hipError_t e = launch_group(g.type, p->d_stages + g.stage0, p->d_first + g.stage0, g.n,
                                          g.tiles, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void free_plan(ct_plan* p) {
    if (!p) return;
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->capture) hipStreamDestroy(p->capture);
    if (p->d_stages) hipFree(p->d_stages);
    if (p->d_first) hipFree(p->d_first);
    if (p->ws) hipFree(p->ws);
    delete p;
}

int check_stream(const ct_stream_desc& d, Geometry* g, bool fused) {
    int rc = resolve(&d.geom, g);
    if (rc != CT_OK) return rc;
    if (d.batch < 1 || d.batch > 65535) return CT_ERR_ARG;
    if (!d.planes || !d.idx || !d.side || !d.steps || !d.out) return CT_ERR_ARG;
    if (!fused && (!d.coeffs || !d.deq)) return CT_ERR_ARG;
    if (d.steps_stride < 0 || (d.steps_stride > 0 && d.steps_stride < g->nsub)) return CT_ERR_ARG;
    return CT_OK;
}

}  // namespace

extern "C" {

int ct_plan_create(const ct_stream_desc* streams, int32_t n, int32_t flags, ct_plan** out) {
    if (!out) return CT_ERR_ARG;
    *out = nullptr;
    if (!streams || n < 1 || n > 4096) return CT_ERR_ARG;
    if (!constants(CT_FILTERS_CDF97).ok || !constants(CT_FILTERS_LEGALL53).ok) return CT_ERR_UNSUPPORTED;
    ct_plan* p = new ct_plan();
    p->streams.assign(streams, streams + n);
    p->geoms.resize(n);
    p->wls.resize(n);
    p->ws_off.resize(n);
    p->grouping.assign(size_t(n) * kMaxLevels, 3);
    size_t total = 0;
    for (int s = 0; s < n; ++s) {
        const int rc = check_stream(streams[s], &p->geoms[s], (flags & CT_PLAN_FUSED) != 0);
        if (rc != CT_OK) {
            free_plan(p);
            return rc;
        }
        p->wls[s] = workspace_layout(p->geoms[s], streams[s].batch);
        p->ws_off[s] = total;
        total += (p->wls[s].total + 255) & ~size_t(255);
    }
    if (hipGetDevice(&p->device) != hipSuccess || hipMalloc(&p->ws, total) != hipSuccess ||
        hipMemset(p->ws, 0, total) != hipSuccess) {
        free_plan(p);
        return CT_ERR_HIP;
    }
    if (hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking) != hipSuccess) {
        free_plan(p);
        return CT_ERR_HIP;
    }
    if (flags & CT_PLAN_AUTOTUNE) {
        const int rc = autotune(p, p->capture);
        if (rc != CT_OK) {
            free_plan(p);
            return rc;
        }
    }
    // per-stream chains
    p->chains.resize(n);
    size_t max_len = 0;
    for (int s = 0; s < n; ++s) {
        const ct_stream_desc& d = streams[s];
        const Geometry& g = p->geoms[s];
        char* ws = p->ws + p->ws_off[s];
        std::vector<StageDesc>& c = p->chains[s];
        const int* grp = &p->grouping[size_t(s) * kMaxLevels];
        int rc = CT_OK;
        if (flags & CT_PLAN_FUSED) {
            // fused encoder and decoder: no dequantised float coefficients;
            // the float coefficients only when the caller asks for them
            const FusedQuant fq{d.idx, d.steps, d.steps_stride, d.side};
            build_transform_chain(g, d.batch, kModeForward, d.planes, d.coeffs, ws, p->wls[s], grp, c, &fq);
            const float* low = d.coeffs ? d.coeffs : reinterpret_cast<const float*>(ws + p->wls[s].low_off);
            rc = build_lowpass_quant_chain(g, d.batch, low, d.coeffs ? g.ncoef : g.low_n, d.steps,
                                           d.steps_stride, d.idx, d.side, ws, p->wls[s], c);
            if (rc == CT_OK)
                build_transform_chain(g, d.batch, kModeInverse, nullptr, d.out, ws, p->wls[s], grp, c, &fq);
        } else {
            build_transform_chain(g, d.batch, kModeForward, d.planes, d.coeffs, ws, p->wls[s], grp, c);
            rc = build_quant_chain(g, d.batch, d.coeffs, d.steps, d.steps_stride, d.idx, d.side, ws,
                                   p->wls[s], c);
            if (rc == CT_OK)
                rc = build_dequant_chain(g, d.batch, d.idx, d.steps, d.steps_stride, d.side, d.deq, c);
            if (rc == CT_OK)
                build_transform_chain(g, d.batch, kModeInverse, d.deq, d.out, ws, p->wls[s], grp, c);
        }
        if (rc != CT_OK) {
            free_plan(p);
            return rc;
        }
        max_len = std::max(max_len, c.size());
    }
    // groups: chain position by chain position, one group per stage type,
    // each group's stages largest first
    std::vector<StageDesc> order;
    std::vector<int> first;
    int64_t items = 0;
    for (size_t w = 0; w < max_len; ++w) {
        for (int type = 0; type < kStNumTypes; ++type) {
            std::vector<int> ids;
            for (int s = 0; s < n; ++s)
                if (p->chains[s].size() > w && p->chains[s][w].type == type) ids.push_back(s);
            if (ids.empty()) continue;
            std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) {
                return p->chains[a][w].ntiles > p->chains[b][w].ntiles;
            });
            ct_plan::Group g{type, int(order.size()), int(ids.size()), 0};
            for (int s : ids) {
                const StageDesc& d = p->chains[s][w];
                first.push_back(g.tiles);
                g.tiles += d.ntiles;
                p->bytes += d.bytes;
                p->alg += d.alg;
                order.push_back(d);
            }
            items += g.tiles;
            p->groups.push_back(g);
        }
    }
    p->nstages = int(order.size());
    if (items >= (int64_t(1) << 31)) {
        free_plan(p);
        return CT_ERR_UNSUPPORTED;
    }
    p->total_items = int(items);
    if (hipMalloc(&p->d_stages, sizeof(StageDesc) * order.size()) != hipSuccess ||
        hipMalloc(&p->d_first, sizeof(int) * first.size()) != hipSuccess ||
        hipMemcpy(p->d_stages, order.data(), sizeof(StageDesc) * order.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->d_first, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice) != hipSuccess) {
        free_plan(p);
        return CT_ERR_HIP;
    }
    if (flags & CT_PLAN_GRAPH) {
        bool ok = hipStreamBeginCapture(p->capture, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) ok = launch_groups(p, p->capture) == hipSuccess;
        hipGraph_t graph = nullptr;
        const bool ended = hipStreamEndCapture(p->capture, &graph) == hipSuccess;
        p->graph = graph;
        ok = ok && ended && graph && hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (!ok) {
            free_plan(p);
            return CT_ERR_HIP;
        }
    }
    *out = p;
    return CT_OK;
}

int ct_plan_run(ct_plan* p, hipStream_t stream) {
    if (!p) return CT_ERR_ARG;
    if (p->exec) {
        CT_PROFILED_ALG("batched_graph", p->bytes, p->alg, hipGraphLaunch(p->exec, stream), stream);
        return CT_OK;
    }
    CT_PROFILED_ALG("batched", p->bytes, p->alg, launch_groups(p, stream), stream);
    return CT_OK;
}

int ct_plan_run_plain(ct_plan* p, hipStream_t stream) {
    if (!p) return CT_ERR_ARG;
    for (const auto& c : p->chains) {
        const int rc = launch_chain(c, stream);
        if (rc != CT_OK) return rc;
    }
    return CT_OK;
}

int ct_plan_info(const ct_plan* p, ct_plan_info_t* info) {
    if (!p || !info) return CT_ERR_ARG;
    info->streams = int32_t(p->streams.size());
    info->stages = p->nstages;
    info->work_items = p->total_items;
    info->launches = int32_t(p->groups.size());
    info->graph = p->exec ? 1 : 0;
    info->autotuned = p->autotuned;
    int n[4] = {0, 0, 0, 0}, h[3] = {0, 0, 0};
    for (size_t s = 0; s < p->streams.size(); ++s)
        for (int j = 0; j < p->geoms[s].J; ++j) {
            const int l = p->geoms[s].l[j];
            const int code = p->grouping[s * kMaxLevels + j];
            int grp = tune_grouping(code);
            if (grp > l - 2) grp = l - 2;       // the same passes as l - 2 levels per pass
            if (l >= 4) n[grp]++;
            if (l >= 3) h[tune_height(code)]++;
        }
    info->levels_single = n[1];
    info->levels_paired = n[2];
    info->levels_triple = n[3];
    info->levels_short_blocks = h[kHeightShort];
    info->levels_tall_blocks = h[kHeightTall];
    info->workspace_bytes = 0;
    for (size_t s = 0; s < p->streams.size(); ++s) info->workspace_bytes += p->wls[s].total;
    return CT_OK;
}

void ct_plan_destroy(ct_plan* p) { free_plan(p); }

}  // extern "C"

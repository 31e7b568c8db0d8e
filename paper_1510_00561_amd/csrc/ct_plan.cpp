// Batched plans: many streams of uneven resolution and LP depth in one graph
// launch (host side).
//
// A plan owns a workspace slice per stream, the stage-descriptor table of
// every stream's chain (forward CT, quantise, dequantise, inverse CT) laid
// out group by group, and, with CT_PLAN_GRAPH, an instantiated HIP graph of
// the group launches. A group is the set of stages of one type at one chain
// position over all streams; its launch covers all their tiles.
//
// With CT_PLAN_AUTOTUNE every stream's geometry goes through the tile-shape
// tuner of the split passes (ct_tune.cpp); without it the plan takes the
// choices an earlier tuning in this process made, else the defaults. No
// choice changes a result.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
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

int autotune(ct_plan* p, hipStream_t st) {
    for (size_t s = 0; s < p->streams.size(); ++s) {
        const int rc = tune_geometry(p->geoms[s], p->streams[s].batch, p->ws + p->ws_off[s], p->wls[s], st,
                                     &p->grouping[s * kMaxLevels]);
        if (rc != CT_OK) return rc;
    }
    p->autotuned = 1;
    return CT_OK;
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
    } else {
        // choices an earlier tuning in this process made for these shapes
        for (int s = 0; s < n; ++s) tuned_codes(p->geoms[s], streams[s].batch, &p->grouping[size_t(s) * kMaxLevels]);
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
    int n[4] = {0, 0, 0, 0}, h[4] = {0, 0, 0, 0};
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
    info->levels_sized_blocks = h[kHeightRows];
    info->workspace_bytes = 0;
    for (size_t s = 0; s < p->streams.size(); ++s) info->workspace_bytes += p->wls[s].total;
    return CT_OK;
}

void ct_plan_destroy(ct_plan* p) { free_plan(p); }

}  // extern "C"

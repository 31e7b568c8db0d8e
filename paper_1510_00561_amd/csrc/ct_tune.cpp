// Tile-shape autotuning of the DFB split passes (host side).
//
// For every LP level with three or more DFB tree levels the tuner times, with
// HIP events, the level's split passes (analysis then synthesis) for every
// combination of
//   * tree levels per streaming pass: one, two or three (up to l - 2), and
//   * row-block height: the host's default, the heights aiming at twice or
//     half as many wavefronts, and explicit heights that cut the tallest
//     parent channel into 2..10 equal blocks,
// and keeps the fastest. Every choice computes the same float32 operations in
// the same order, so none changes a result. Choices are cached in a JSON file
// keyed by device architecture and shape (CT_AUTOTUNE_CACHE, default
// $HOME/.cache/ct_autotune.json) and kept in a per-process table keyed by
// device and shape, which the per-call entry points (ct_forward, ct_encode,
// ...) read when they build their stage chains.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "ct_internal.h"
#include "ct_kernels.h"
#include "ct_plan_internal.h"

namespace ct {
namespace {

// ---------------------------------------------------------------- JSON cache
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
    if (!f) return;   // no writable cache: the choices stay in this process only
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

// ---------------------------------------------------------------- per-process table
using ShapeKey = std::tuple<int, int, int, int, int>;   // device, R_j, C_j, l, batch
std::mutex g_table_mu;
std::map<ShapeKey, int>& table() {
    static std::map<ShapeKey, int> t;
    return t;
}

// ---------------------------------------------------------------- timing
void split_passes(int l, int grouping, int* first, int* count, int* ng) {
    *ng = 0;
    for (int t = 3; t <= l;) {
        const int c = t + grouping - 1 <= l ? grouping : l - t + 1;
        first[*ng] = t;
        count[*ng] = c;
        ++*ng;
        t += c;
    }
}

// Time the DFB split passes (analysis then synthesis) of one LP level shape
// with the given tune code, using workspace buffers as scratch.
float time_level_splits(int Rj, int Cj, int l, int batch, int code, float* A, float* B, float* D, int64_t plane,
                        hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
    int first[4], count[4], ng = 0;
    split_passes(l, tune_grouping(code), first, count, &ng);
    static hipError_t (*const ana[3])(const SplitArgs&, Lift, int, hipStream_t) = {
        launch_dfb_split_analysis, launch_dfb_split2_analysis, launch_dfb_split3_analysis};
    static hipError_t (*const syn[3])(const SplitArgs&, Lift, int, hipStream_t) = {
        launch_dfb_split_synthesis, launch_dfb_split2_synthesis, launch_dfb_split3_synthesis};
    Lift L{{-1.5f, -0.05f, 0.88f, 0.44f}, 1};
    auto args = [&](int gi, const float* parent, float* child) {
        SplitArgs a;
        memset(&a, 0, sizeof(a));
        a.t = first[gi];
        a.Rj = Rj;
        a.Cj = Cj;
        a.parent = parent;
        a.parent_plane = plane;
        a.child = child;
        a.child_plane = plane;
        a.plane_elems = int64_t(Rj) * Cj;
        a.bh = split_block_rows(a, batch, count[gi], tune_height(code), tune_rows(code));
        return a;
    };
    auto run = [&]() -> bool {
        float* cur = A;
        float* other = B;
        for (int gi = 0; gi < ng; ++gi) {
            if (ana[count[gi] - 1](args(gi, cur, gi == ng - 1 ? D : other), L, batch, st) != hipSuccess) return false;
            std::swap(cur, other);
        }
        cur = A;
        other = B;
        for (int gi = ng - 1; gi >= 0; --gi) {
            if (syn[count[gi] - 1](args(gi, gi == ng - 1 ? D : other, cur), L, batch, st) != hipSuccess) return false;
            std::swap(cur, other);
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

// The codes tried for a level: every grouping that differs for this depth
// (up to l - 2 levels per pass) at every candidate height.
std::vector<int> candidates(int Rj, int Cj, int l) {
    std::vector<int> rows;
    const int tallest = (Rj > Cj ? Rj : Cj) >> 1;     // parent rows of the first pass
    for (int nb = 2; nb <= 10; ++nb) {
        int r = (tallest + nb - 1) / nb;
        r = (r + 7) / 8 * 8;
        if (r < 32 || r > 248) continue;
        bool dup = false;
        for (int x : rows) dup = dup || x == r;
        if (!dup) rows.push_back(r);
    }
    std::vector<int> codes;
    for (int grp = 1; grp <= 3 && grp <= l - 2; ++grp) {
        for (int hm = kHeightDefault; hm <= kHeightTall; ++hm) codes.push_back(tune_code(grp, hm));
        for (int r : rows) codes.push_back(tune_code(grp, kHeightRows, r));
    }
    return codes;
}

}  // namespace

bool valid_tune(int code) {
    const int g = tune_grouping(code), h = tune_height(code), r = tune_rows(code);
    if (code < 0 || (code >> 16) != 0 || (code & 0xc0) != 0 || g < 1 || g > 3) return false;
    return h == kHeightRows ? (r >= 32 && r <= 1020) : r == 0;
}

void tuned_codes(const Geometry& g, int batch, int* codes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = -1;
    std::lock_guard<std::mutex> lock(g_table_mu);
    const std::map<ShapeKey, int>& t = table();
    for (int j = 1; j <= kMaxLevels; ++j) {
        codes[j - 1] = kDefaultTune;
        if (j > g.J || t.empty()) continue;
        auto it = t.find(ShapeKey{dev, g.R >> (j - 1), g.C >> (j - 1), g.l[j - 1], batch});
        if (it != t.end()) codes[j - 1] = it->second;
    }
}

int tune_geometry(const Geometry& g, int batch, char* ws, const Workspace& w, hipStream_t st, int* codes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CT_ERR_HIP;
    std::map<std::string, int> cache = load_cache();
    const std::string arch = arch_name(dev);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return CT_ERR_HIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return CT_ERR_HIP;
    }
    bool dirty = false;
    int rc = CT_OK;
    for (int j = 1; j <= g.J && rc == CT_OK; ++j) {
        const int l = g.l[j - 1];
        codes[j - 1] = kDefaultTune;
        if (l < 3) continue;    // no split pass
        const int Rj = g.R >> (j - 1), Cj = g.C >> (j - 1);
        char key[160];
        snprintf(key, sizeof(key), "%s|split_tune|%dx%d|l%d|b%d", arch.c_str(), Rj, Cj, l, batch);
        auto it = cache.find(key);
        int choice = kDefaultTune;
        if (it != cache.end() && valid_tune(it->second)) {
            choice = it->second;
        } else {
            float* A = reinterpret_cast<float*>(ws + w.a_off);
            float* B = reinterpret_cast<float*>(ws + w.b_off);
            float* D = reinterpret_cast<float*>(ws + w.d_off);
            const int64_t plane = int64_t(g.R) * g.C;
            float best = -1.f;
            for (int code : candidates(Rj, Cj, l)) {
                const float ms = time_level_splits(Rj, Cj, l, batch, code, A, B, D, plane, st, e0, e1);
                if (ms < 0) {
                    rc = CT_ERR_HIP;
                    break;
                }
                if (best < 0 || ms < best) {
                    best = ms;
                    choice = code;
                }
            }
            if (rc != CT_OK) break;
            cache[key] = choice;
            dirty = true;
        }
        codes[j - 1] = choice;
        std::lock_guard<std::mutex> lock(g_table_mu);
        table()[ShapeKey{dev, Rj, Cj, l, batch}] = choice;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (dirty) save_cache(cache);
    return rc;
}

}  // namespace ct

extern "C" {

int ct_autotune(const ct_geom* geom, int32_t batch, void* ws, size_t ws_bytes, hipStream_t stream) {
    ct::Geometry g;
    if (!geom || batch < 0 || batch > 65535) return CT_ERR_ARG;
    int rc = ct::resolve(geom, &g);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!ws) return CT_ERR_ARG;
    const ct::Workspace w = ct::workspace_layout(g, batch);
    if (ws_bytes < w.total) return CT_ERR_WORKSPACE;
    int codes[ct::kMaxLevels];
    return ct::tune_geometry(g, batch, static_cast<char*>(ws), w, stream, codes);
}

int ct_autotune_clear(void) {
    std::lock_guard<std::mutex> lock(ct::g_table_mu);
    ct::table().clear();
    return CT_OK;
}

}  // extern "C"

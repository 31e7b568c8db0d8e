// C ABI of the P-frame motion compensation (paper section 3.7), the zero-run
// coder (section 3.8) and the host DEFLATE stage (section 3.9): validation
// and tables on the host, device passes in ct_codec.hip. The run-length
// decoder and DEFLATE / INFLATE are host code, as the paper runs them on the
// CPU (section 3.7: the serial stages).
#include <hip/hip_runtime.h>
#include <zlib.h>

#include <cstdlib>
#include <cstring>
#include <vector>

#include "ct_codec.h"
#include "ct_plan_internal.h"

namespace {

bool fault_injected() {
    const char* f = getenv("CT_FAULT_INJECT");
    return f && strcmp(f, "launch") == 0;
}

int log2i(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Level table of a geometry from its subband table (storage positions: the
// lowpass, then levels J..1).
int level_table(const ct::Geometry& g, ct::codec::LevelTable* T, int* nrows) {
    using ct::codec::kMaxDirs;
    std::vector<ct_subband> tab(g.nsub);
    ct::subband_table(g, tab.data(), g.nsub);
    memset(T, 0, sizeof(*T));
    T->J = g.J;
    T->R = g.R;
    T->C = g.C;
    T->ncoef = g.ncoef;
    if (g.ncoef >= (int64_t(1) << 30)) return CT_ERR_UNSUPPORTED;
    T->nsub_l[0] = 1;
    T->sub0[0] = 0;
    int s = 1;
    for (int p = 1; p <= g.J; ++p) {
        const int j = g.J + 1 - p;
        const int nd = g.dirs[j - 1];
        T->off[p] = tab[s].offset;
        T->sub0[j] = s;
        T->nsub_l[j] = nd;
        T->nh[j] = nd / 2;
        const ct_subband& h = tab[s];
        const ct_subband& v = tab[s + nd / 2];
        if (h.transposed || !v.transposed || nd > kMaxDirs) return CT_ERR_GEOM;
        T->rows_h[j] = h.rows;
        T->cols_h[j] = h.cols;
        T->rows_v[j] = v.rows;
        T->cols_v[j] = v.cols;
        T->lsh1_h[j] = log2i(h.s1);
        T->lsh2_h[j] = log2i(h.s2);
        T->lsh1_v[j] = log2i(v.s1);
        T->lsh2_v[j] = log2i(v.s2);
        for (int k = 0; k < nd; ++k) {
            T->o1[j][k] = int8_t(tab[s + k].o1);
            T->o2[j][k] = int8_t(tab[s + k].o2);
        }
        s += nd;
    }
    T->off[0] = 0;
    T->off[g.J + 1] = g.ncoef;
    int r = 0;
    for (int p = 0; p <= g.J; ++p) {
        T->row0[p] = r;
        if (p == 0) {
            r += g.R >> g.J;
        } else {
            const int j = g.J + 1 - p;
            r += T->nh[j] * T->rows_h[j] + (T->nsub_l[j] - T->nh[j]) * T->rows_v[j];
        }
    }
    T->row0[g.J + 1] = r;
    *nrows = r;
    return CT_OK;
}

int geometry(const ct_geom* geom, int32_t batch, ct::Geometry* g) {
    if (!geom || batch < 0 || batch > 65535) return CT_ERR_ARG;
    return ct::resolve(geom, g);
}

// Natural row length and count of component s, and whether it is coded.
struct Comp {
    int rows, cols;
    bool transposed, coded;
    int64_t offset;
};

// Offsets of a plane's stream: non-negative and non-decreasing, so that every
// component lies inside the sub_off[n] symbols the caller holds. Checked in
// full before any symbol is touched.
bool offsets_ok(const int32_t* sub_off, int n) {
    if (sub_off[0] < 0) return false;
    for (int s = 0; s < n; ++s)
        if (sub_off[s + 1] < sub_off[s]) return false;
    return true;
}

std::vector<Comp> components(const ct::Geometry& g, int p_frame) {
    std::vector<ct_subband> tab(g.nsub);
    ct::subband_table(g, tab.data(), g.nsub);
    std::vector<Comp> c(g.nsub);
    for (int s = 0; s < g.nsub; ++s)
        c[s] = Comp{tab[s].rows, tab[s].cols, tab[s].transposed != 0, p_frame != 0 || s > 0, tab[s].offset};
    return c;
}

}  // namespace

extern "C" {

int ct_mc_residual(const ct_geom* geom, int32_t batch, int32_t n, const int16_t* cur, const int16_t* prev,
                   const int16_t* mv, int32_t nby, int32_t nbx, int32_t mv_group, int32_t inverse,
                   int16_t* out, hipStream_t stream) {
    ct::Geometry g;
    int rc = geometry(geom, batch, &g);
    if (rc != CT_OK) return rc;
    if (n < 1 || n > CT_MAX_CHROMA_FACTOR || nby < 1 || nbx < 1 || mv_group < 1) return CT_ERR_ARG;
    if (batch == 0) return CT_OK;
    if (!cur || !prev || !mv || !out) return CT_ERR_ARG;
    if (out == prev) return CT_ERR_ARG;
    ct::codec::MCArgs a;
    int nrows = 0;
    rc = level_table(g, &a.T, &nrows);
    if (rc != CT_OK) return rc;
    if (fault_injected()) return CT_ERR_HIP;
    a.cur = cur;
    a.prev = prev;
    a.mv = mv;
    a.out = out;
    a.batch = batch;
    a.n = n;
    a.nby = nby;
    a.nbx = nbx;
    a.group = mv_group;
    a.inverse = inverse != 0;
    const double bytes = 6.0 * double(batch) * double(g.ncoef);
    CT_PROFILED("mc_residual", bytes, ct::codec::launch_mc(a, stream), stream);
    return CT_OK;
}

int ct_rle_workspace_bytes(const ct_geom* geom, int32_t batch, size_t* bytes) {
    if (bytes) *bytes = 0;
    if (!bytes) return CT_ERR_ARG;
    ct::Geometry g;
    int rc = geometry(geom, batch, &g);
    if (rc != CT_OK) return rc;
    ct::codec::LevelTable T;
    int nrows = 0;
    rc = level_table(g, &T, &nrows);
    if (rc != CT_OK) return rc;
    *bytes = size_t(2) * size_t(batch) * size_t(nrows) * sizeof(int32_t);
    return CT_OK;
}

int ct_rle_encode(const ct_geom* geom, int32_t batch, const int16_t* idx, int32_t p_frame, int16_t* symbols,
                  int32_t* sub_off, void* ws, size_t ws_bytes, hipStream_t stream) {
    ct::Geometry g;
    int rc = geometry(geom, batch, &g);
    if (rc != CT_OK) return rc;
    if (batch == 0) return CT_OK;
    if (!idx || !symbols || !sub_off || !ws) return CT_ERR_ARG;
    ct::codec::RLEArgs a;
    int nrows = 0;
    rc = level_table(g, &a.T, &nrows);
    if (rc != CT_OK) return rc;
    // natural rows longer than an int16 run cannot be coded
    for (int j = 1; j <= g.J; ++j)
        if (a.T.cols_h[j] > 32767 || a.T.cols_v[j] > 32767) return CT_ERR_UNSUPPORTED;
    if ((g.C >> g.J) > 32767) return CT_ERR_UNSUPPORTED;
    const size_t need = size_t(2) * size_t(batch) * size_t(nrows) * sizeof(int32_t);
    if (ws_bytes < need) return CT_ERR_WORKSPACE;
    if (fault_injected()) return CT_ERR_HIP;
    a.idx = idx;
    a.sym = symbols;
    a.sub_off = sub_off;
    a.rowcnt = static_cast<int32_t*>(ws);
    a.rowoff = a.rowcnt + size_t(batch) * nrows;
    a.batch = batch;
    a.nsub = g.nsub;
    a.nrows = nrows;
    a.p_frame = p_frame != 0;
    const double bytes = 2.0 * double(batch) * double(g.ncoef);   // the indices, read once (symbols: data-dependent)
    CT_PROFILED("rle_encode", bytes, ct::codec::launch_rle(a, stream), stream);
    return CT_OK;
}

int ct_rle_decode_host(const ct_geom* geom, const int16_t* symbols, const int32_t* sub_off, int32_t p_frame,
                       int16_t* idx) {
    ct::Geometry g;
    const int rc = geometry(geom, 1, &g);
    if (rc != CT_OK) return rc;
    if (!symbols || !sub_off || !idx) return CT_ERR_ARG;
    if (!offsets_ok(sub_off, g.nsub)) return CT_ERR_ARG;
    const std::vector<Comp> comps = components(g, p_frame);
    for (int s = 0; s < g.nsub; ++s) {
        const Comp& c = comps[s];
        int64_t pos = sub_off[s];
        const int64_t end = sub_off[s + 1];
        if (pos < 0 || end < pos) return CT_ERR_ARG;
        int16_t* dst = idx + c.offset;
        if (!c.coded) {
            if (end - pos != int64_t(c.rows) * c.cols) return CT_ERR_ARG;
            memcpy(dst, symbols + pos, sizeof(int16_t) * size_t(c.rows) * c.cols);
            continue;
        }
        for (int i = 0; i < c.rows; ++i) {
            int k = 0;
            while (k < c.cols) {
                if (pos >= end) return CT_ERR_ARG;
                const int16_t v = symbols[pos++];
                int run = 1;
                if (v == 0) {
                    if (pos >= end) return CT_ERR_ARG;
                    run = symbols[pos++];
                    if (run < 1 || k + run > c.cols) return CT_ERR_ARG;
                }
                for (int r = 0; r < run; ++r, ++k) {
                    const int64_t e = c.transposed ? int64_t(k) * c.rows + i : int64_t(i) * c.cols + k;
                    dst[e] = v;
                }
            }
        }
        if (pos != end) return CT_ERR_ARG;
    }
    return CT_OK;
}

int ct_deflate_host(const int16_t* symbols, const int32_t* sub_off, int32_t nsub, int32_t mode, int32_t level,
                    uint8_t* out, size_t cap, uint32_t* comp_bytes, size_t* total) {
    if (total) *total = 0;
    if (!symbols || !sub_off || !comp_bytes || !total || nsub < 1 || (mode != 0 && mode != 1)) return CT_ERR_ARG;
    if (level < 0 || level > 9 || (cap > 0 && !out)) return CT_ERR_ARG;
    if (!offsets_ok(sub_off, nsub)) return CT_ERR_ARG;
    const int parts = mode == 0 ? nsub : 1;
    size_t used = 0;
    for (int s = 0; s < parts; ++s) {
        const int64_t a = mode == 0 ? sub_off[s] : sub_off[0];
        const int64_t b = mode == 0 ? sub_off[s + 1] : sub_off[nsub];
        if (a < 0 || b < a) return CT_ERR_ARG;
        const uLong src_len = uLong(b - a) * sizeof(int16_t);   // little-endian int16 on this host
        uLongf dst_len = compressBound(src_len);
        if (used + dst_len > cap) return CT_ERR_WORKSPACE;
        if (compress2(out + used, &dst_len, reinterpret_cast<const Bytef*>(symbols + a), src_len, level) != Z_OK)
            return CT_ERR_UNSUPPORTED;
        comp_bytes[s] = uint32_t(dst_len);
        used += dst_len;
    }
    *total = used;
    return CT_OK;
}

int ct_inflate_host(const uint8_t* in, const uint32_t* comp_bytes, const int32_t* sub_off, int32_t nsub,
                    int32_t mode, int16_t* symbols) {
    if (!in || !comp_bytes || !sub_off || !symbols || nsub < 1 || (mode != 0 && mode != 1)) return CT_ERR_ARG;
    if (!offsets_ok(sub_off, nsub)) return CT_ERR_ARG;
    const int parts = mode == 0 ? nsub : 1;
    size_t used = 0;
    for (int s = 0; s < parts; ++s) {
        const int64_t a = mode == 0 ? sub_off[s] : sub_off[0];
        const int64_t b = mode == 0 ? sub_off[s + 1] : sub_off[nsub];
        if (a < 0 || b < a) return CT_ERR_ARG;
        uLongf dst_len = uLongf(b - a) * sizeof(int16_t);
        if (uncompress(reinterpret_cast<Bytef*>(symbols + a), &dst_len, in + used, comp_bytes[s]) != Z_OK ||
            dst_len != uLongf(b - a) * sizeof(int16_t))
            return CT_ERR_ARG;
        used += comp_bytes[s];
    }
    return CT_OK;
}

}  // extern "C"

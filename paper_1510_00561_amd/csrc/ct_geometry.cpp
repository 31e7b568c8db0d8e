// Geometry, layout and workspace of the contourlet transform (host only).
//
// Paper: section 3.3 (every LP level halves the resolution; the stream holds
// the coarsest lowpass and the directional subbands of every scale, coarse
// scales first so that finer ones can be dropped), section 2.1 (2^l wedge
// subbands per DFB). Boundary handling, padding, tree geometry and the
// packed order are the reading documented in ct.h.
#include <string.h>

#include "ct_internal.h"

namespace ct {
namespace {

int ilog2_pow2(int v) {
    if (v <= 0 || (v & (v - 1))) return -1;
    int r = 0;
    while ((1 << r) < v) ++r;
    return r;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Leaf {
    int o1, o2;
};

// Offsets of the DFB channels down the tree, in level-image coordinates.
//
// Tree level 2 puts the four channels on the cosets of 2Z^2:
//   horizontal a=-1 -> (0,1), horizontal a=0 -> (1,0),
//   vertical a=0 -> (0,0),    vertical a=-1 -> (1,1).
// A split at tree level t >= 3 (m = t - 2) of a channel with parameter a and
// offset o uses v1 = (2a, -2^m) (vertical) or (-2^m, 2a) (horizontal); the
// even child (a' = 2a + 1) keeps o, the odd child (a' = 2a) moves to o + v1.
// Offsets are reduced modulo the child lattice diag(2, 2^(m+1)) (vertical) or
// diag(2^(m+1), 2) (horizontal).
void walk(bool vertical, int a, int o1, int o2, int t, int l, Leaf* leaves) {
    if (t > l) {
        int q = 1 << (l - 2);
        int k = vertical ? (1 << (l - 1)) + (q - 1 - a) : a + q;
        leaves[k] = Leaf{o1, o2};
        return;
    }
    int m = t - 2;
    int d1 = vertical ? 2 : (1 << (m + 1));
    int d2 = vertical ? (1 << (m + 1)) : 2;
    int v1r = vertical ? 2 * a : -(1 << m);
    int v1c = vertical ? -(1 << m) : 2 * a;
    auto mod = [](int x, int n) { return ((x % n) + n) % n; };
    walk(vertical, 2 * a + 1, mod(o1, d1), mod(o2, d2), t + 1, l, leaves);
    walk(vertical, 2 * a, mod(o1 + v1r, d1), mod(o2 + v1c, d2), t + 1, l, leaves);
}

void dfb_leaves(int l, Leaf* leaves) {
    walk(false, -1, 0, 1, 3, l, leaves);
    walk(false, 0, 1, 0, 3, l, leaves);
    walk(true, 0, 0, 0, 3, l, leaves);
    walk(true, -1, 1, 1, 3, l, leaves);
}

}  // namespace

int resolve(const ct_geom* g, Geometry* out) {
    if (!g || !out) return CT_ERR_ARG;
    Geometry r;
    if (g->levels < 1 || g->levels > kMaxLevels) return CT_ERR_GEOM;
    if (g->height <= 0 || g->width <= 0) return CT_ERR_GEOM;
    r.H = g->height;
    r.W = g->width;
    r.J = g->levels;
    if (g->filters != CT_FILTERS_CDF97 && g->filters != CT_FILTERS_LEGALL53) return CT_ERR_GEOM;
    if (g->recon != CT_RECON_DUAL && g->recon != CT_RECON_BURT_ADELSON) return CT_ERR_GEOM;
    r.filters = g->filters;
    r.recon = g->recon;
    r.e = r.J;
    for (int j = 0; j < r.J; ++j) {
        int lj = ilog2_pow2(g->dirs[j]);
        if (lj < 2 || lj > 6) return CT_ERR_GEOM;
        r.dirs[j] = g->dirs[j];
        r.l[j] = lj;
        int need = (j + 1) + lj - 2;
        if (need > r.e) r.e = need;
    }
    const int step = 1 << r.e;
    if (r.H < step || r.W < step) return CT_ERR_GEOM;
    if (r.H > 32768 || r.W > 32768) return CT_ERR_GEOM;
    r.R = (r.H + step - 1) / step * step;
    r.C = (r.W + step - 1) / step * step;
    // Levels with three or more tree levels run split stages on channels of
    // R_j / 2 or C_j / 2 columns, which they move in column pairs: the choice
    // of e (>= j + 1 there) keeps R_j and C_j multiples of 4.
    for (int j = 1; j <= r.J; ++j)
        if (r.l[j - 1] >= 3 && (((r.R >> (j - 1)) & 3) || ((r.C >> (j - 1)) & 3))) return CT_ERR_GEOM;
    r.low_n = int64_t(r.R >> r.J) * (r.C >> r.J);
    int64_t off = r.low_n;
    r.nsub = 1;
    for (int j = r.J; j >= 1; --j) {
        r.level_off[j] = off;
        off += int64_t(r.R >> (j - 1)) * (r.C >> (j - 1));
        r.nsub += r.dirs[j - 1];
    }
    r.ncoef = off;
    if (r.ncoef >= (int64_t(1) << 31)) return CT_ERR_GEOM;
    *out = r;
    return CT_OK;
}

void subband_table(const Geometry& g, ct_subband* table, int cap) {
    int n = 0;
    auto put = [&](const ct_subband& s) {
        if (n < cap) table[n] = s;
        ++n;
    };
    ct_subband low;
    memset(&low, 0, sizeof(low));
    low.level = g.J + 1;
    low.k = -1;
    low.rows = g.R >> g.J;
    low.cols = g.C >> g.J;
    low.offset = 0;
    low.s1 = low.s2 = 1;
    put(low);
    for (int j = g.J; j >= 1; --j) {
        const int l = g.l[j - 1];
        const int Rj = g.R >> (j - 1), Cj = g.C >> (j - 1);
        const int nb = 1 << l, half = nb / 2;
        Leaf leaves[kMaxDirs];
        dfb_leaves(l, leaves);
        int64_t off = g.level_off[j];
        for (int k = 0; k < nb; ++k) {
            ct_subband s;
            memset(&s, 0, sizeof(s));
            const bool vertical = k >= half;
            s.level = j;
            s.k = k;
            s.s1 = vertical ? 2 : half;
            s.s2 = vertical ? half : 2;
            s.rows = Rj / s.s1;
            s.cols = Cj / s.s2;
            s.offset = off;
            s.o1 = leaves[k].o1;
            s.o2 = leaves[k].o2;
            s.transposed = vertical ? 1 : 0;
            off += int64_t(s.rows) * s.cols;
            put(s);
        }
    }
}

void dfb_scale_exponents(int l, int* out) {
    // positions after tree level 2: [H a=-1, H a=0, V a=0, V a=-1]
    // exponents: H is the odd child at tree level 1 (-1), V the even (+1);
    // at tree level 2 the even children are H a=0 and V a=0.
    int cur[kMaxDirs], nxt[kMaxDirs];
    cur[0] = -2;
    cur[1] = 0;
    cur[2] = 2;
    cur[3] = 0;
    for (int t = 3; t <= l; ++t) {
        const int np = 1 << (t - 1), hp = np / 2;
        for (int p = 0; p < np; ++p) {
            // horizontal parent p: children 2p (odd, a'=2a), 2p+1 (even)
            // vertical parent p: children 2p (even, a'=2a+1), 2p+1 (odd)
            const bool vertical = p >= hp;
            nxt[2 * p] = cur[p] + (vertical ? +1 : -1);
            nxt[2 * p + 1] = cur[p] + (vertical ? -1 : +1);
        }
        memcpy(cur, nxt, sizeof(int) * (2 * np));
    }
    memcpy(out, cur, sizeof(int) * (1 << l));
}

Workspace workspace_layout(const Geometry& g, int batch) {
    Workspace w;
    size_t off = 0;
    const size_t B = size_t(batch);
    for (int j = 1; j < g.J; ++j) {
        w.c_off[j] = off;
        off = align256(off + B * size_t(g.R >> j) * size_t(g.C >> j) * sizeof(float));
    }
    const size_t plane = size_t(g.R) * size_t(g.C) * sizeof(float);
    w.d_off = off;
    off = align256(off + B * plane);
    w.a_off = off;
    off = align256(off + B * plane);
    w.b_off = off;
    off = align256(off + B * plane);
    // channels of LP levels 2..J, apart from level 1's, so that level 1's
    // split passes can run beside the coarser levels
    w.a2_off = off;
    off = align256(off + (g.J > 1 ? B * plane / 4 : 0));
    w.b2_off = off;
    off = align256(off + (g.J > 1 ? B * plane / 4 : 0));
    w.part_off = off;
    off = align256(off + B * kMaxPart * 2 * sizeof(float));
    w.low_off = off;
    off = align256(off + B * size_t(g.low_n) * sizeof(float));
    w.total = off;
    return w;
}

}  // namespace ct

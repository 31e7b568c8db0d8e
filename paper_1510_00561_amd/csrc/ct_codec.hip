// P-frame motion compensation (paper section 3.7) and zero-run coding
// (section 3.8) of the quantised CT components, for gfx950.
//
// Motion compensation is one pass over the indices, one wavefront per stored
// row of a component, four consecutive elements per lane: every element finds
// the 16 x 16 block of the luminance pixel it sits on, that block's vector
// mapped to the component's sample spacing (rounded, halves away from zero),
// and subtracts (or, for the decoder, adds) the previous plane's element at
// the displaced position, modulo the component's size and modulo 2^16.
// HBM-bound: 2 bytes read, 2 gathered (mostly within the lines of nearby
// rows) and 2 written per element.
//
// The zero-run coder is a stream compaction in three passes:
//   1. symbols per natural row: rows stored contiguously (the lowpass, the
//      horizontal-cone subbands) take one wavefront each, lanes along the
//      row, four elements per lane; rows of the transposed vertical-cone
//      subbands are stored columns, so one wavefront takes 64 of them, one
//      per lane, and walks down the stored rows with coalesced loads;
//   2. per plane, an exclusive scan of the row counts (one workgroup per
//      plane) gives every row's symbol offset and every component's offset;
//   3. symbols: the same decomposition as pass 1. Along a contiguous row,
//      lanes take four consecutive elements each; a row's symbol positions
//      come from a prefix sum of the per-element symbol counts (1 for a
//      non-zero value, 2 for the first zero of a run), and the element that
//      ends a run writes its length next to the run's 0, found from a prefix
//      maximum of the last non-zero position.
#include "ct_codec.h"

namespace ct {
namespace codec {
namespace {

constexpr int NT = 256;

__device__ __forceinline__ int pmod(int a, int n) {
    const int r = a % n;
    return r < 0 ? r + n : r;
}

// Storage position p (0 = lowpass, then levels J..1) -> level index (0 =
// lowpass, else the LP level j).
__device__ __forceinline__ int level_of_pos(const LevelTable& T, int p) { return p == 0 ? 0 : T.J + 1 - p; }

__device__ __forceinline__ int find_pos(const LevelTable& T, int64_t e) {
    int p = 0;
    while (p < T.J && e >= T.off[p + 1]) ++p;
    return p;
}

// floor(x / b) for 0 <= x < 2^22 and 1 <= b < 2^22, with rb = 1/b: the float
// quotient is within one of the true one, and one correction each way makes
// it exact.
__device__ __forceinline__ int udiv_small(int x, int b, float rb) {
    int q = int(float(x) * rb);
    if ((q + 1) * b <= x) ++q;
    if (q * b > x) --q;
    return q;
}

// a / b rounded to the nearest integer, halves away from zero: floor((2|a| +
// b) / (2b)) with the sign of a (|a| <= 32768, b < 2^20).
__device__ __forceinline__ int round_div_fast(int a, int b2, float rb2) {
    const int q = udiv_small(2 * abs(a) + (b2 >> 1), b2, rb2);
    return a < 0 ? -q : q;
}

// (t mod n) for the displaced index t of an element, usually within one
// period of the component.
__device__ __forceinline__ int wrap(int t, int n) {
    if (t >= 0 && t < n) return t;
    if (t < 0 && t >= -n) return t + n;
    if (t >= n && t < 2 * n) return t - n;
    return pmod(t, n);
}

// One wavefront per stored row of one component of one plane. The row's
// component, its natural row (or, for the transposed vertical-cone subbands,
// natural column), the sample spacing and the block row (column) are the
// same for the whole wavefront; lanes step along the row.
struct MCItem {
    int64_t start;      // first element of the stored row within the plane
    int len;            // elements along the stored row
    bool tr;            // transposed subband: the row is a natural column
    int fixed;          // natural row (row-major) or natural column (transposed)
    int rows, cols;     // natural size of the component
    int f, s1, s2, o1, o2;   // pixel = f (o + s (i, k))
    int64_t base;       // first element of the component
};

__device__ MCItem mc_item(const LevelTable& T, const int* item0, int it, int n, bool* ok) {
    MCItem m;
    int p = 0;
    while (p <= T.J && it >= item0[p + 1]) ++p;
    *ok = p <= T.J;
    if (!*ok) return m;
    const int lv = level_of_pos(T, p);
    int w = it - item0[p];
    m.tr = false;
    if (lv == 0) {
        m.rows = T.R >> T.J;
        m.cols = T.C >> T.J;
        m.base = 0;
        m.fixed = w;
        m.start = int64_t(w) * m.cols;
        m.len = m.cols;
        m.f = n << T.J;
        m.s1 = m.s2 = 1;
        m.o1 = m.o2 = 0;
        return m;
    }
    const int sz = T.rows_h[lv] * T.cols_h[lv];
    const int nhr = T.nh[lv] * T.rows_h[lv];
    m.f = n << (lv - 1);
    int kk;
    if (w < nhr) {
        kk = w / T.rows_h[lv];
        const int i = w - kk * T.rows_h[lv];
        m.rows = T.rows_h[lv];
        m.cols = T.cols_h[lv];
        m.fixed = i;
        m.len = m.cols;
        m.s1 = 1 << T.lsh1_h[lv];
        m.s2 = 1 << T.lsh2_h[lv];
        m.base = T.off[p] + int64_t(kk) * sz;
        m.start = m.base + int64_t(i) * m.cols;
    } else {
        w -= nhr;
        const int kv = w / T.cols_v[lv], k = w - kv * T.cols_v[lv];
        kk = T.nh[lv] + kv;
        m.tr = true;
        m.rows = T.rows_v[lv];
        m.cols = T.cols_v[lv];
        m.fixed = k;
        m.len = m.rows;
        m.s1 = 1 << T.lsh1_v[lv];
        m.s2 = 1 << T.lsh2_v[lv];
        m.base = T.off[p] + int64_t(kk) * sz;
        m.start = m.base + int64_t(k) * m.rows;
    }
    m.o1 = T.o1[lv][kk];
    m.o2 = T.o2[lv][kk];
    return m;
}

struct MCItems {
    int item0[kMaxLevels + 3];
};

MCItems mc_items_of(const LevelTable& T) {
    MCItems it;
    it.item0[0] = 0;
    for (int p = 0; p <= T.J; ++p) {
        const int lv = p == 0 ? 0 : T.J + 1 - p;
        const int n = lv == 0 ? (T.R >> T.J)
                              : T.nh[lv] * T.rows_h[lv] + (T.nsub_l[lv] - T.nh[lv]) * T.cols_v[lv];
        it.item0[p + 1] = it.item0[p] + n;
    }
    for (int p = T.J + 2; p < kMaxLevels + 3; ++p) it.item0[p] = it.item0[T.J + 1];
    return it;
}

__global__ __launch_bounds__(NT) void mc_kernel(MCArgs A, MCItems IT) {
    const LevelTable& T = A.T;
    const int per = IT.item0[T.J + 1];
    const int gw = __builtin_amdgcn_readfirstlane(int(blockIdx.x) * (NT / 64) + int(threadIdx.x >> 6));
    if (gw >= per * A.batch) return;
    const int b = gw / per;
    bool ok;
    const MCItem m = mc_item(T, IT.item0, gw - b * per, A.n, &ok);
    if (!ok) return;
    const int lane = threadIdx.x & 63;
    const int16_t* cur = A.cur + int64_t(b) * T.ncoef;
    const int16_t* prev = A.prev + int64_t(b) * T.ncoef;
    int16_t* out = A.out + int64_t(b) * T.ncoef;
    const int16_t* mv = A.mv + int64_t(b / A.group) * A.nby * A.nbx * 2;
    const int sy = m.f * m.s1, sx = m.f * m.s2;            // sample spacing in pixels
    const float rby = 1.f / float(2 * sy), rbx = 1.f / float(2 * sx);
    // the fixed coordinate's block and pixel
    const int fixed_px = m.f * ((m.tr ? m.o2 : m.o1) + (m.tr ? m.s2 : m.s1) * m.fixed);
    const int fixed_blk = m.tr ? min(fixed_px >> 4, A.nbx - 1) : min(fixed_px >> 4, A.nby - 1);
    // lanes take four consecutive elements each: one 8-byte load and store of
    // the row when it is 8-byte aligned (the gathers stay per element)
    const int16_t* crow = cur + m.start;
    int16_t* orow = out + m.start;
    const bool vec = ((reinterpret_cast<uintptr_t>(crow) | reinterpret_cast<uintptr_t>(orow)) & 7) == 0;
    const bool mv4 = (reinterpret_cast<uintptr_t>(mv) & 3) == 0;
    const int vo = m.tr ? m.o1 : m.o2, vs = m.tr ? m.s1 : m.s2;
    for (int e0 = 4 * lane; e0 < m.len; e0 += 256) {
        const bool full = vec && e0 + 4 <= m.len;
        int cv[4];
        if (full) {
            const int2 w = *reinterpret_cast<const int2*>(crow + e0);
            cv[0] = int16_t(w.x & 0xffff);
            cv[1] = int16_t(uint32_t(w.x) >> 16);
            cv[2] = int16_t(w.y & 0xffff);
            cv[3] = int16_t(uint32_t(w.y) >> 16);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) cv[q] = e0 + q < m.len ? int(crow[e0 + q]) : 0;
        }
        int r[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = min(e0 + q, m.len - 1);   // past the row end: a valid element, not stored
            // the varying coordinate: natural column (row-major) or row (transposed)
            const int px = m.f * (vo + vs * e);
            const int vb = m.tr ? min(px >> 4, A.nby - 1) : min(px >> 4, A.nbx - 1);
            const int by = m.tr ? vb : fixed_blk, bx = m.tr ? fixed_blk : vb;
            const int16_t* v = mv + (by * A.nbx + bx) * 2;
            int dy, dx;
            if (mv4) {
                const int w = *reinterpret_cast<const int*>(v);
                dy = int16_t(w & 0xffff);
                dx = int16_t(uint32_t(w) >> 16);
            } else {
                dy = v[0];
                dx = v[1];
            }
            const int i = m.tr ? e : m.fixed, k = m.tr ? m.fixed : e;
            const int i2 = wrap(i + round_div_fast(dy, 2 * sy, rby), m.rows);
            const int k2 = wrap(k + round_div_fast(dx, 2 * sx, rbx), m.cols);
            const int64_t src = m.base + (m.tr ? int64_t(k2) * m.rows + i2 : int64_t(i2) * m.cols + k2);
            const int pv = prev[src];
            r[q] = A.inverse ? cv[q] + pv : cv[q] - pv;   // modulo 2^16 on the store
        }
        if (full) {
            int2 w;
            w.x = int((uint32_t(r[0]) & 0xffffu) | (uint32_t(r[1]) << 16));
            w.y = int((uint32_t(r[2]) & 0xffffu) | (uint32_t(r[3]) << 16));
            *reinterpret_cast<int2*>(orow + e0) = w;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (e0 + q < m.len) orow[e0 + q] = int16_t(r[q]);
        }
    }
}

// ---------------------------------------------------------------- zero runs

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int wave_incl_sum(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ int wave_incl_max(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o) v = max(v, t);
    }
    return v;
}

// What one wavefront item of a plane covers.
struct Item {
    bool valid;
    bool contiguous;     // one row, lanes along it; else up to 64 transposed rows, one per lane
    bool coded;          // zero runs coded (else the row is copied unchanged)
    int64_t start;       // element offset (within the plane) of the row, or of the stored block
    int len;             // row length (contiguous) / natural row length (transposed)
    int rows_v;          // transposed: natural rows of the subband (stored row stride)
    int i0;              // transposed: first natural row of the item
    int row;             // row id of the (first) natural row
};

// Items of storage position p: the lowpass rows; or, for a level, nh * rows_h
// contiguous rows, then (nsub - nh) * ceil(rows_v / 64) transposed groups.
__device__ Item item_of(const LevelTable& T, const int* item0, int it, int p_frame) {
    Item r;
    r.valid = false;
    int p = 0;
    while (p <= T.J && it >= item0[p + 1]) ++p;
    if (p > T.J) return r;
    r.valid = true;
    const int lv = level_of_pos(T, p);
    int w = it - item0[p];
    if (lv == 0) {
        const int cols = T.C >> T.J;
        r.contiguous = true;
        r.coded = p_frame != 0;
        r.start = int64_t(w) * cols;
        r.len = cols;
        r.row = T.row0[p] + w;
        return r;
    }
    r.coded = true;
    const int sz = T.rows_h[lv] * T.cols_h[lv];
    const int nhr = T.nh[lv] * T.rows_h[lv];
    if (w < nhr) {
        r.contiguous = true;
        const int kk = w / T.rows_h[lv], i = w - kk * T.rows_h[lv];
        r.start = T.off[p] + int64_t(kk) * sz + int64_t(i) * T.cols_h[lv];
        r.len = T.cols_h[lv];
        r.row = T.row0[p] + w;
        return r;
    }
    w -= nhr;
    const int groups = (T.rows_v[lv] + 63) / 64;
    const int kv = w / groups, g = w - kv * groups;
    r.contiguous = false;
    r.start = T.off[p] + int64_t(T.nh[lv] + kv) * sz;
    r.len = T.cols_v[lv];
    r.rows_v = T.rows_v[lv];
    r.i0 = 64 * g;
    r.row = T.row0[p] + nhr + kv * T.rows_v[lv] + r.i0;
    return r;
}

struct ItemTable {
    int item0[kMaxLevels + 3];
};

// Elements e0 .. e0 + 3 of a row of `len` (1 past the end: a non-zero value
// that ends any run and is never coded); one 8-byte load when the row is
// 8-byte aligned and the four are inside it.
__device__ __forceinline__ void load4(const int16_t* x, int e0, int len, bool aligned, int* v) {
    if (aligned && e0 + 4 <= len) {
        const int2 w = *reinterpret_cast<const int2*>(x + e0);
        v[0] = int16_t(w.x & 0xffff);
        v[1] = int16_t(uint32_t(w.x) >> 16);
        v[2] = int16_t(w.y & 0xffff);
        v[3] = int16_t(uint32_t(w.y) >> 16);
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = e0 + q < len ? int(x[e0 + q]) : 1;
    }
}

__global__ __launch_bounds__(NT) void rle_count_kernel(RLEArgs A, ItemTable IT) {
    const LevelTable& T = A.T;
    const int per = IT.item0[T.J + 1];
    const int gw = int(blockIdx.x) * (NT / 64) + int(threadIdx.x >> 6);
    if (gw >= per * A.batch) return;
    const int b = gw / per;
    const Item m = item_of(T, IT.item0, gw - b * per, A.p_frame);
    if (!m.valid) return;
    const int lane = lane_id();
    const int16_t* x = A.idx + int64_t(b) * T.ncoef + m.start;
    int32_t* cnt = A.rowcnt + int64_t(b) * A.nrows;
    if (m.contiguous) {
        int c = 0;
        if (!m.coded) {
            c = m.len;
        } else {
            const bool al = (reinterpret_cast<uintptr_t>(x) & 7) == 0;
            int carry = 1;                         // before the row: "non-zero"
            for (int c0 = 0; c0 < m.len; c0 += 256) {
                const int e0 = c0 + 4 * lane;
                int v[4];
                load4(x, e0, m.len, al, v);
                const int up = __shfl_up(v[3], 1, 64);
                int pv = lane == 0 ? carry : up;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (e0 + q < m.len) c += v[q] != 0 ? 1 : (pv != 0 ? 2 : 0);
                    pv = v[q];
                }
                carry = __shfl(v[3], 63, 64);
            }
            c = wave_incl_sum(c);
            c = __shfl(c, 63, 64);
        }
        if (lane == 0) cnt[m.row] = c;
    } else {
        const int i = m.i0 + lane;
        if (i < m.rows_v) {
            int c = 0;
            bool pnz = true;
            for (int r = 0; r < m.len; ++r) {
                const int v = x[int64_t(r) * m.rows_v + i];
                c += v != 0 ? 1 : (pnz ? 2 : 0);
                pnz = v != 0;
            }
            cnt[m.row + lane] = c;
        }
    }
}

// One workgroup per plane: exclusive scan of the plane's row counts, and the
// symbol offset of every component.
constexpr int SCAN_NT = 1024;
__global__ __launch_bounds__(SCAN_NT) void rle_scan_kernel(RLEArgs A) {
    __shared__ int part[SCAN_NT / 64];
    __shared__ int tot;
    const LevelTable& T = A.T;
    const int b = blockIdx.x;
    const int32_t* cnt = A.rowcnt + int64_t(b) * A.nrows;
    int32_t* off = A.rowoff + int64_t(b) * A.nrows;
    const int chunk = (A.nrows + SCAN_NT - 1) / SCAN_NT;
    const int r0 = min(A.nrows, int(threadIdx.x) * chunk), r1 = min(A.nrows, r0 + chunk);
    int s = 0;
    for (int r = r0; r < r1; ++r) s += cnt[r];
    const int incl = wave_incl_sum(s);
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 63) part[wv] = incl;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wv; ++w) before += part[w];
    if (threadIdx.x == SCAN_NT - 1) tot = before + incl;
    int run = before + incl - s;
    for (int r = r0; r < r1; ++r) {
        off[r] = run;
        run += cnt[r];
    }
    __syncthreads();
    // component offsets: component s is subband k of storage position p
    int32_t* so = A.sub_off + int64_t(b) * (A.nsub + 1);
    for (int sb = threadIdx.x; sb < A.nsub; sb += SCAN_NT) {
        int p = 0;
        while (p < T.J && sb >= T.sub0[level_of_pos(T, p + 1)]) ++p;
        const int lv = level_of_pos(T, p);
        const int k = sb - T.sub0[lv];
        int row = T.row0[p];
        if (lv > 0) row += k < T.nh[lv] ? k * T.rows_h[lv] : T.nh[lv] * T.rows_h[lv] + (k - T.nh[lv]) * T.rows_v[lv];
        so[sb] = row < A.nrows ? off[row] : tot;
    }
    if (threadIdx.x == 0) so[A.nsub] = tot;
}

// Zero-run symbols of one natural row of `len` elements at stride `ld`,
// written from dst[pos] on.
__device__ __forceinline__ void rle_column(const int16_t* x, int len, int ld, int16_t* dst, int pos) {
    bool in_run = false;
    int run_tok = 0, run_len = 0;
    for (int r = 0; r < len; ++r) {
        const int v = x[int64_t(r) * ld];
        if (v != 0) {
            if (in_run) {
                dst[run_tok + 1] = int16_t(run_len);
                in_run = false;
            }
            dst[pos++] = int16_t(v);
        } else {
            if (!in_run) {
                in_run = true;
                run_tok = pos;
                dst[pos] = 0;
                pos += 2;
                run_len = 0;
            }
            ++run_len;
        }
    }
    if (in_run) dst[run_tok + 1] = int16_t(run_len);
}

__global__ __launch_bounds__(NT) void rle_write_kernel(RLEArgs A, ItemTable IT) {
    const LevelTable& T = A.T;
    const int per = IT.item0[T.J + 1];
    const int gw = int(blockIdx.x) * (NT / 64) + int(threadIdx.x >> 6);
    if (gw >= per * A.batch) return;
    const int b = gw / per;
    const Item m = item_of(T, IT.item0, gw - b * per, A.p_frame);
    if (!m.valid) return;
    const int lane = lane_id();
    const int16_t* x = A.idx + int64_t(b) * T.ncoef + m.start;
    const int32_t* off = A.rowoff + int64_t(b) * A.nrows;
    int16_t* out = A.sym + int64_t(b) * 2 * T.ncoef;
    if (m.contiguous) {
        int pos = off[m.row];
        if (!m.coded) {
            for (int e = lane; e < m.len; e += 64) out[pos + e] = x[e];
            return;
        }
        const bool al = (reinterpret_cast<uintptr_t>(x) & 7) == 0;
        int carry = 1;            // element before the chunk (before the row: non-zero)
        int lastnz = -1;          // last non-zero position before the chunk
        for (int c0 = 0; c0 < m.len; c0 += 256) {
            const int e0 = c0 + 4 * lane;
            int v[4];
            load4(x, e0, m.len, al, v);
            const int up = __shfl_up(v[3], 1, 64);
            const int dn = __shfl_down(v[0], 1, 64);
            const int pv0 = lane == 0 ? carry : up;
            // the element after e0 + 3
            const int nv3 = lane == 63 ? (e0 + 4 < m.len ? int(x[e0 + 4]) : 1) : (e0 + 4 < m.len ? dn : 1);
            int sc[4], tot = 0, lnz = -1;
            int pv = pv0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool in = e0 + q < m.len;
                sc[q] = in ? (v[q] != 0 ? 1 : (pv != 0 ? 2 : 0)) : 0;
                tot += sc[q];
                if (in && v[q] != 0) lnz = e0 + q;
                pv = v[q];
            }
            const int incl = wave_incl_sum(tot);
            const int nzi = wave_incl_max(lnz);
            const int nzu = __shfl_up(nzi, 1, 64);
            int nz = max(lastnz, lane == 0 ? -1 : nzu);   // last non-zero before e0
            int p = pos + incl - tot;
            pv = pv0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = e0 + q;
                if (e < m.len) {
                    const int nv = q < 3 ? v[q + 1] : nv3;
                    if (v[q] != 0) {
                        out[p] = int16_t(v[q]);
                        nz = e;
                    } else {
                        if (pv != 0) out[p] = 0;                     // a run starts here
                        if (nv != 0) {                               // and ends here
                            const int start = nz + 1;
                            out[start == e ? p + 1 : p - 1] = int16_t(e - start + 1);
                        }
                    }
                }
                p += sc[q];
                pv = v[q];
            }
            pos += __shfl(incl, 63, 64);
            carry = __shfl(v[3], 63, 64);
            lastnz = max(lastnz, __shfl(nzi, 63, 64));
        }
    } else {
        // one natural row per lane; the symbols go straight to the stream
        // (staging the 64 rows' symbols in LDS and copying them out
        // coalesced measured slower: 470 against 370 us for the coder at
        // 1080p)
        const int i = m.i0 + lane;
        if (i < m.rows_v) rle_column(x + i, m.len, m.rows_v, out, off[m.row + lane]);
    }
}

ItemTable items_of(const LevelTable& T) {
    ItemTable it;
    it.item0[0] = 0;
    for (int p = 0; p <= T.J; ++p) {
        const int lv = p == 0 ? 0 : T.J + 1 - p;
        int n;
        if (lv == 0) n = T.R >> T.J;
        else n = T.nh[lv] * T.rows_h[lv] + (T.nsub_l[lv] - T.nh[lv]) * ((T.rows_v[lv] + 63) / 64);
        it.item0[p + 1] = it.item0[p] + n;
    }
    for (int p = T.J + 2; p < kMaxLevels + 3; ++p) it.item0[p] = it.item0[T.J + 1];
    return it;
}

}  // namespace

hipError_t launch_mc(const MCArgs& a, hipStream_t st) {
    if (a.batch == 0) return hipSuccess;
    const MCItems it = mc_items_of(a.T);
    const int64_t waves = int64_t(it.item0[a.T.J + 1]) * a.batch;
    mc_kernel<<<unsigned((waves + NT / 64 - 1) / (NT / 64)), NT, 0, st>>>(a, it);
    return hipGetLastError();
}

hipError_t launch_rle(const RLEArgs& a, hipStream_t st) {
    if (a.batch == 0) return hipSuccess;
    const ItemTable it = items_of(a.T);
    const int64_t waves = int64_t(it.item0[a.T.J + 1]) * a.batch;
    const unsigned blocks = unsigned((waves + NT / 64 - 1) / (NT / 64));
    rle_count_kernel<<<blocks, NT, 0, st>>>(a, it);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    rle_scan_kernel<<<a.batch, SCAN_NT, 0, st>>>(a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    rle_write_kernel<<<blocks, NT, 0, st>>>(a, it);
    return hipGetLastError();
}

}  // namespace codec
}  // namespace ct

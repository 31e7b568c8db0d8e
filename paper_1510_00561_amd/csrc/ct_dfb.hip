// Directional filter bank kernels for gfx950.
//
// Paper section 2.1: the DFB splits each LP bandpass image into 2^l wedge
// subbands with the 9-7 filters. Every tree node is a quincunx fan filter
// bank (the 9-7 pair with cos(w) replaced by the fan kernel
// K = (S_v2 + S_-v2 - S_v1 - S_-v1)/4 of the node's lattice basis). Here it
// runs as the lifting factorisation of the 9-7 pair: four steps
//     odd += c0 N(even); even += c1 N(odd); odd += c2 N(even); even += c3 N(odd)
// with the neighbour sum N = 2K. The per-level scaling (even * zeta,
// odd / zeta) is deferred: a channel's scale is the product over its path
// and is applied once where its final subband is stored (or loaded, in the
// synthesis direction).
//
// Tree levels 1 and 2 (dfb12 kernels) act on the full level image:
//   level 1: basis (1,0), (0,1); parity n1 + n2; N(x)[n] = x[n+(0,1)] +
//            x[n-(0,1)] - x[n+(1,0)] - x[n-(1,0)], halved;
//   level 2: both cones at once: parity n2; diagonal neighbours
//            N(x)[n] = x[n+(-1,1)] + x[n+(1,-1)] - x[n+(1,1)] - x[n-(1,1)], halved.
// A 256-thread workgroup lifts a 64 x 64 tile with an 8-pixel halo in LDS;
// each step only updates the region the final interior still depends on.
//
// Tree levels t >= 3 (split kernels) act on compact channel arrays. A
// horizontal channel on diag(2^(t-2), 2) Z^2 with parameter a is split along
// rows: its neighbours are at compact offsets (-1, a), (-1, a+1) and their
// mirrors. Vertical channels are kept transposed, which turns their
// column split into the same row split, so one kernel serves both cones and
// every access runs along the contiguous axis. In the sheared frame
// Q[i, k] = P[i, k - a i] the neighbourhood becomes the fixed stencil
//     N[i][k] = Q[i-1][k+1] + Q[i+1][k-1] - Q[i-1][k] - Q[i+1][k], halved,
// so a rectangular LDS tile in Q (a parallelogram in P, loaded row by row
// with a per-row start offset) needs only a 4-row, 4-column halo.
#include "ct_kernels.h"

namespace ct {
namespace {

constexpr int NT = 256;
__device__ __forceinline__ int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

// ---------------------------------------------------------------- dfb12
constexpr int QT = 64, QH = 8;
constexpr int QN = QT + 2 * QH;   // 80
constexpr int QLD = QN + 1;

// One lifting step of tree level 1 over rows/cols [m, QN - m).
__device__ __forceinline__ void step_cross(float (*T)[QLD], int par, float coef, int m) {
    const int span = QN - 2 * m;            // even
    const int half = span / 2;
    for (int idx = threadIdx.x; idx < span * half; idx += NT) {
        const int rr = idx / half, j = idx - rr * half;
        const int r = m + rr;
        // column with (r + c) & 1 == par, first candidate m or m + 1
        const int c = m + 2 * j + ((r + m + par) & 1);
        T[r][c] += coef * (T[r][c + 1] + T[r][c - 1] - T[r + 1][c] - T[r - 1][c]);
    }
}

// One lifting step of tree level 2 over rows/cols [m, QN - m).
__device__ __forceinline__ void step_diag(float (*T)[QLD], int par, float coef, int m) {
    const int span = QN - 2 * m;
    const int half = span / 2;
    for (int idx = threadIdx.x; idx < span * half; idx += NT) {
        const int rr = idx / half, j = idx - rr * half;
        const int r = m + rr;
        const int c = m + 2 * j + ((m + par) & 1);
        T[r][c] += coef * (T[r - 1][c + 1] + T[r + 1][c - 1] - T[r + 1][c + 1] - T[r - 1][c - 1]);
    }
}

__global__ __launch_bounds__(NT) void dfb12_analysis_kernel(CView d, int R, int C, Quad out,
                                                            Lift L) {
    __shared__ float T[QN][QLD];
    const int gx = (C + QT - 1) / QT, gy = (R + QT - 1) / QT;
    const int Lt = xcd_remap(blockIdx.x, gridDim.x);
    const int n0 = ((Lt / gx) % gy) * QT, m0 = (Lt % gx) * QT, b = Lt / (gx * gy);
    const float* dp = d.p + b * d.plane;
    for (int idx = threadIdx.x; idx < QN * QN; idx += NT) {
        const int r = idx / QN, c = idx - r * QN;
        T[r][c] = dp[int64_t(wrap(n0 - QH + r, R)) * d.ld + wrap(m0 - QH + c, C)];
    }
    __syncthreads();
    int m = 1;
    for (int s = 0; s < 4; ++s, ++m) {
        step_cross(T, (L.first_odd + s) & 1, 0.5f * L.c[s], m);
        __syncthreads();
    }
    for (int s = 0; s < 4; ++s, ++m) {
        step_diag(T, (L.first_odd + s) & 1, 0.5f * L.c[s], m);
        __syncthreads();
    }
    const int Rh = R >> 1, Ch = C >> 1;
    // horizontal channels, row major (R/2) x (C/2): quad 0 = coset (0,1), 1 = (1,0)
    for (int idx = threadIdx.x; idx < 2 * (QT / 2) * (QT / 2); idx += NT) {
        const int q = idx / ((QT / 2) * (QT / 2));
        const int rem = idx - q * (QT / 2) * (QT / 2);
        const int i = rem / (QT / 2), k = rem - i * (QT / 2);
        const int pr = q == 0 ? 0 : 1, pc = q == 0 ? 1 : 0;
        const int gi = (n0 >> 1) + i, gk = (m0 >> 1) + k;
        if (gi < Rh && gk < Ch)
            out.p[q][b * out.plane + int64_t(gi) * Ch + gk] = out.scale[q] * T[QH + 2 * i + pr][QH + 2 * k + pc];
    }
    // vertical channels, transposed (C/2) x (R/2): quad 2 = coset (0,0), 3 = (1,1)
    for (int idx = threadIdx.x; idx < 2 * (QT / 2) * (QT / 2); idx += NT) {
        const int q = 2 + idx / ((QT / 2) * (QT / 2));
        const int rem = idx - (q - 2) * (QT / 2) * (QT / 2);
        const int k = rem / (QT / 2), i = rem - k * (QT / 2);
        const int p = q == 2 ? 0 : 1;
        const int gi = (n0 >> 1) + i, gk = (m0 >> 1) + k;
        if (gi < Rh && gk < Ch)
            out.p[q][b * out.plane + int64_t(gk) * Rh + gi] = out.scale[q] * T[QH + 2 * i + p][QH + 2 * k + p];
    }
}

__global__ __launch_bounds__(NT) void dfb12_synthesis_kernel(Quad in, int R, int C, View d,
                                                             Lift L) {
    __shared__ float T[QN][QLD];
    const int gx = (C + QT - 1) / QT, gy = (R + QT - 1) / QT;
    const int Lt = xcd_remap(blockIdx.x, gridDim.x);
    const int n0 = ((Lt / gx) % gy) * QT, m0 = (Lt % gx) * QT, b = Lt / (gx * gy);
    const int Rh = R >> 1, Ch = C >> 1;
    constexpr int HN = QN / 2;   // 40 compact samples per axis
    // horizontal channels (row major): lanes run along compact columns
    for (int idx = threadIdx.x; idx < 2 * HN * HN; idx += NT) {
        const int q = idx / (HN * HN);
        const int rem = idx - q * HN * HN;
        const int i = rem / HN, k = rem - i * HN;
        const int pr = q == 0 ? 0 : 1, pc = q == 0 ? 1 : 0;
        const int gi = wrap((n0 >> 1) - QH / 2 + i, Rh), gk = wrap((m0 >> 1) - QH / 2 + k, Ch);
        T[2 * i + pr][2 * k + pc] = in.scale[q] * in.p[q][b * in.plane + int64_t(gi) * Ch + gk];
    }
    // vertical channels (transposed): lanes run along compact rows
    for (int idx = threadIdx.x; idx < 2 * HN * HN; idx += NT) {
        const int q = 2 + idx / (HN * HN);
        const int rem = idx - (q - 2) * HN * HN;
        const int k = rem / HN, i = rem - k * HN;
        const int p = q == 2 ? 0 : 1;
        const int gi = wrap((n0 >> 1) - QH / 2 + i, Rh), gk = wrap((m0 >> 1) - QH / 2 + k, Ch);
        T[2 * i + p][2 * k + p] = in.scale[q] * in.p[q][b * in.plane + int64_t(gk) * Rh + gi];
    }
    __syncthreads();
    int m = 1;
    for (int s = 0; s < 4; ++s, ++m) {
        step_diag(T, (L.first_odd + s) & 1, 0.5f * L.c[s], m);
        __syncthreads();
    }
    for (int s = 0; s < 4; ++s, ++m) {
        step_cross(T, (L.first_odd + s) & 1, 0.5f * L.c[s], m);
        __syncthreads();
    }
    float* dp = d.p + b * d.plane;
    for (int idx = threadIdx.x; idx < QT * QT; idx += NT) {
        const int i = idx / QT, j = idx - i * QT;
        const int gr = n0 + i, gc = m0 + j;
        if (gr < R && gc < C) dp[int64_t(gr) * d.ld + gc] = T[QH + i][QH + j];
    }
}

// ---------------------------------------------------------------- split
constexpr int ST_R = 32, ST_C = 64, SH = 4;
constexpr int SN_R = ST_R + 2 * SH;    // 40
constexpr int SN_C = ST_C + 2 * SH;    // 72
constexpr int SLD = SN_C + 1;

// Tiles of one horizontal and one vertical parent channel at tree level t.
__device__ __forceinline__ void split_tile_counts(const SplitArgs& A, int& th, int& tv) {
    const int t = A.t;
    auto tiles = [](int nr, int nc) { return ((nr + ST_R - 1) / ST_R) * ((nc + ST_C - 1) / ST_C); };
    th = tiles(A.Rj >> (t - 2), A.Cj >> 1);
    tv = tiles(A.Cj >> (t - 2), A.Rj >> 1);
}

struct SplitGeom {
    int nr, nc;             // parent array size
    int a;                  // shear parameter
    int64_t parent_off;     // element offset of the parent channel in a plane
    int64_t even_off, odd_off;  // offsets of the even-row and odd-row children
    int even_pos, odd_pos;  // child channel positions (for the scale table)
    int rtiles, ctiles;
};

__device__ __forceinline__ SplitGeom split_geom(const SplitArgs& A, int pp) {
    SplitGeom g;
    const int t = A.t;
    const int np = 1 << (t - 1), hp = np >> 1;   // parents at tree level t - 1
    const bool vertical = pp >= hp;
    const int q = 1 << (t - 3);
    if (!vertical) {
        g.a = pp - q;
        g.nr = A.Rj >> (t - 2);
        g.nc = A.Cj >> 1;
        g.odd_pos = 2 * pp;            // a' = 2a
        g.even_pos = 2 * pp + 1;       // a' = 2a + 1
    } else {
        g.a = q - 1 - (pp - hp);
        g.nr = A.Cj >> (t - 2);
        g.nc = A.Rj >> 1;
        g.even_pos = 2 * pp;
        g.odd_pos = 2 * pp + 1;
    }
    const int64_t psize = A.plane_elems >> (t - 1);
    const int64_t csize = A.plane_elems >> t;
    g.parent_off = pp * psize;
    g.even_off = g.even_pos * csize;
    g.odd_off = g.odd_pos * csize;
    g.rtiles = (g.nr + ST_R - 1) / ST_R;
    g.ctiles = (g.nc + ST_C - 1) / ST_C;
    return g;
}

// Logical block -> (parent channel, tile within it, plane). Per plane the
// horizontal parents come first, each with th tiles, then the vertical ones.
__device__ __forceinline__ void split_decode(const SplitArgs& A, int L, int& pp, int& tile, int& b) {
    int th, tv;
    split_tile_counts(A, th, tv);
    const int nh = 1 << (A.t - 2);
    const int per_plane = nh * (th + tv);
    b = L / per_plane;
    int rem = L - b * per_plane;
    if (rem < nh * th) {
        pp = rem / th;
        tile = rem - pp * th;
    } else {
        rem -= nh * th;
        const int v = rem / tv;
        pp = nh + v;
        tile = rem - v * tv;
    }
}

// Lifting step on rows of parity `par` in the sheared tile, rows/cols [m, N - m).
__device__ __forceinline__ void step_shear(float (*Q)[SLD], int par, float coef, int m) {
    const int rows = (SN_R - 2 * m) / 2;   // rows of the given parity
    const int cols = SN_C - 2 * m;
    for (int idx = threadIdx.x; idx < rows * cols; idx += NT) {
        const int rr = idx / cols, cc = idx - rr * cols;
        const int r = m + 2 * rr + ((m + par) & 1);
        const int c = m + cc;
        Q[r][c] += coef * (Q[r - 1][c + 1] + Q[r + 1][c - 1] - Q[r - 1][c] - Q[r + 1][c]);
    }
}

__global__ __launch_bounds__(NT) void split_analysis_kernel(SplitArgs A, Lift L) {
    __shared__ float Q[SN_R][SLD];
    int pp, tile, b;
    split_decode(A, xcd_remap(blockIdx.x, gridDim.x), pp, tile, b);
    const SplitGeom g = split_geom(A, pp);
    const int tr = tile / g.ctiles, tc = tile - tr * g.ctiles;
    const int r0 = tr * ST_R, k0 = tc * ST_C;
    const float* P = A.parent + b * A.parent_plane + g.parent_off;
    for (int idx = threadIdx.x; idx < SN_R * SN_C; idx += NT) {
        const int r = idx / SN_C, c = idx - r * SN_C;
        const int i = r0 - SH + r;                 // unwrapped row (sets the shear)
        const int k = k0 - SH + c;
        Q[r][c] = P[int64_t(wrap(i, g.nr)) * g.nc + wrap(k - g.a * i, g.nc)];
    }
    __syncthreads();
    for (int s = 0; s < 4; ++s) {
        step_shear(Q, (L.first_odd + s) & 1, 0.5f * L.c[s], s + 1);
        __syncthreads();
    }
    float* ce = A.child + b * A.child_plane + g.even_off;
    float* co = A.child + b * A.child_plane + g.odd_off;
    const float se = A.use_scale ? A.scale[g.even_pos] : 1.f;
    const float so = A.use_scale ? A.scale[g.odd_pos] : 1.f;
    for (int idx = threadIdx.x; idx < ST_R * ST_C; idx += NT) {
        const int r = idx / ST_C, c = idx - r * ST_C;
        const int i = r0 + r, k = k0 + c;
        if (i >= g.nr || k >= g.nc) continue;
        const int col = wrap(k - g.a * i, g.nc);
        const float v = Q[SH + r][SH + c];
        if ((i & 1) == 0)
            ce[int64_t(i >> 1) * g.nc + col] = se * v;
        else
            co[int64_t(i >> 1) * g.nc + col] = so * v;
    }
}

__global__ __launch_bounds__(NT) void split_synthesis_kernel(SplitArgs A, Lift L) {
    __shared__ float Q[SN_R][SLD];
    int pp, tile, b;
    split_decode(A, xcd_remap(blockIdx.x, gridDim.x), pp, tile, b);
    const SplitGeom g = split_geom(A, pp);
    const int tr = tile / g.ctiles, tc = tile - tr * g.ctiles;
    const int r0 = tr * ST_R, k0 = tc * ST_C;
    // here `parent` points at the children (input) and `child` at the parent (output)
    const float* ce = A.parent + b * A.parent_plane + g.even_off;
    const float* co = A.parent + b * A.parent_plane + g.odd_off;
    const float se = A.use_scale ? A.scale[g.even_pos] : 1.f;
    const float so = A.use_scale ? A.scale[g.odd_pos] : 1.f;
    for (int idx = threadIdx.x; idx < SN_R * SN_C; idx += NT) {
        const int r = idx / SN_C, c = idx - r * SN_C;
        const int i = r0 - SH + r;
        const int k = k0 - SH + c;
        const int ii = wrap(i, g.nr);
        const int col = wrap(k - g.a * i, g.nc);
        Q[r][c] = (ii & 1) ? so * co[int64_t(ii >> 1) * g.nc + col]
                           : se * ce[int64_t(ii >> 1) * g.nc + col];
    }
    __syncthreads();
    for (int s = 0; s < 4; ++s) {
        step_shear(Q, (L.first_odd + s) & 1, 0.5f * L.c[s], s + 1);
        __syncthreads();
    }
    float* P = A.child + b * A.child_plane + g.parent_off;
    for (int idx = threadIdx.x; idx < ST_R * ST_C; idx += NT) {
        const int r = idx / ST_C, c = idx - r * ST_C;
        const int i = r0 + r, k = k0 + c;
        if (i >= g.nr || k >= g.nc) continue;
        P[int64_t(i) * g.nc + wrap(k - g.a * i, g.nc)] = Q[SH + r][SH + c];
    }
}

// ---------------------------------------------------------------- split pair
// Two consecutive tree levels t and t+1 in one pass, in the sheared frame Q of
// the level-(t-1) parent. After the level-t split the even child (rows
// i = 2i') and the odd child (i = 2i' + 1) live in their own sheared frames
//   even: Q'[i', k'] = Q[2i', k' - i']     odd: Q'[i', k'] = Q[2i' + 1, k' + a]
// so their level-(t+1) neighbourhoods, written in Q, are
//   even rows: N = Q[i-2][k+2] + Q[i+2][k-2] - Q[i-2][k+1] - Q[i+2][k-1]
//   odd rows:  N = Q[i-2][k+1] + Q[i+2][k-1] - Q[i-2][k]   - Q[i+2][k]
// (halved), and the sub-parity of row i in its child is (i >> 1) & 1. The four
// grandchildren are the rows i = 0, 1, 2, 3 (mod 4); every sample keeps the
// parent's natural column k - a i. A 64 x 64 tile needs a 12-row,
// 12-column halo: 4 for level t and 8 for level t+1.
constexpr int PT = 64, PH = 12;
constexpr int PN = PT + 2 * PH;     // 88
constexpr int PLD = PN + 1;

__device__ __forceinline__ void step_pair_first(float (*Q)[PLD], int par, float coef, int m) {
    const int rows = (PN - 2 * m) / 2, cols = PN - 2 * m;
    const int first = m + ((m + par) & 1);
    for (int idx = threadIdx.x; idx < rows * cols; idx += NT) {
        const int rr = idx / cols, cc = idx - rr * cols;
        const int r = first + 2 * rr, c = m + cc;
        Q[r][c] += coef * ((Q[r - 1][c + 1] + Q[r + 1][c - 1]) - (Q[r - 1][c] + Q[r + 1][c]));
    }
}

// rows with (r >> 1) & 1 == par in [m, PN - m); m even
__device__ __forceinline__ void step_pair_second(float (*Q)[PLD], int par, float coef, int m) {
    const int rows = (PN - 2 * m) / 2, cols = PN - 2 * m;
    const int first = m + ((((m >> 1) & 1) == par) ? 0 : 2);
    for (int idx = threadIdx.x; idx < rows * cols; idx += NT) {
        const int rr = idx / cols, cc = idx - rr * cols;
        const int r = first + 4 * (rr >> 1) + (rr & 1), c = m + cc;
        const int e = (~r) & 1;    // 1 for the even child: extra column shift
        Q[r][c] += coef * ((Q[r - 2][c + 1 + e] + Q[r + 2][c - 1 - e]) -
                           (Q[r - 2][c + e] + Q[r + 2][c - e]));
    }
}

// Channel position of grandchild (row class i & 3) of parent pp.
__device__ __forceinline__ int grandchild_pos(bool vertical, int pp, int cls) {
    // horizontal: even child = 2pp+1 (its even/odd children 4pp+3 / 4pp+2),
    //             odd child  = 2pp   (its even/odd children 4pp+1 / 4pp)
    // vertical:   even child = 2pp   (4pp / 4pp+1), odd child = 2pp+1 (4pp+2 / 4pp+3)
    const int h = (cls & 1) ? 1 - (cls >> 1) : 3 - (cls >> 1);   // 3, 1, 2, 0
    const int v = ((cls & 1) << 1) | (cls >> 1);                 // 0, 2, 1, 3
    return 4 * pp + (vertical ? v : h);
}

__device__ __forceinline__ void pair_decode(const SplitArgs& A, int L, int& pp, int& tile, int& b,
                                            int& ctiles) {
    const int t = A.t;
    auto cnt = [](int nr, int nc, int& ct) {
        ct = (nc + PT - 1) / PT;
        return ((nr + PT - 1) / PT) * ct;
    };
    int cth, ctv;
    const int th = cnt(A.Rj >> (t - 2), A.Cj >> 1, cth);
    const int tv = cnt(A.Cj >> (t - 2), A.Rj >> 1, ctv);
    const int nh = 1 << (t - 2);
    const int per_plane = nh * (th + tv);
    b = L / per_plane;
    int rem = L - b * per_plane;
    if (rem < nh * th) {
        pp = rem / th;
        tile = rem - pp * th;
        ctiles = cth;
    } else {
        rem -= nh * th;
        const int v = rem / tv;
        pp = nh + v;
        tile = rem - v * tv;
        ctiles = ctv;
    }
}

__global__ __launch_bounds__(NT) void split2_analysis_kernel(SplitArgs A, Lift L) {
    __shared__ float Q[PN][PLD];
    int pp, tile, b, ctiles;
    pair_decode(A, xcd_remap(blockIdx.x, gridDim.x), pp, tile, b, ctiles);
    const SplitGeom g = split_geom(A, pp);
    const bool vertical = pp >= (1 << (A.t - 2));
    const int r0 = (tile / ctiles) * PT, k0 = (tile % ctiles) * PT;
    const float* P = A.parent + b * A.parent_plane + g.parent_off;
    for (int idx = threadIdx.x; idx < PN * PN; idx += NT) {
        const int r = idx / PN, c = idx - r * PN;
        const int i = r0 - PH + r, k = k0 - PH + c;
        Q[r][c] = P[int64_t(wrap(i, g.nr)) * g.nc + wrap(k - g.a * i, g.nc)];
    }
    __syncthreads();
    for (int s = 0; s < 4; ++s) {
        step_pair_first(Q, (L.first_odd + s) & 1, 0.5f * L.c[s], s + 1);
        __syncthreads();
    }
    for (int s = 0; s < 4; ++s) {
        step_pair_second(Q, (L.first_odd + s) & 1, 0.5f * L.c[s], 6 + 2 * s);
        __syncthreads();
    }
    const int64_t gsize = A.plane_elems >> (A.t + 1);
    float* out = A.child + b * A.child_plane;
    for (int idx = threadIdx.x; idx < PT * PT; idx += NT) {
        const int r = idx / PT, c = idx - r * PT;
        const int i = r0 + r, k = k0 + c;
        if (i >= g.nr || k >= g.nc) continue;
        const int pos = grandchild_pos(vertical, pp, i & 3);
        const float sc = A.use_scale ? A.scale[pos] : 1.f;
        out[pos * gsize + int64_t(i >> 2) * g.nc + wrap(k - g.a * i, g.nc)] = sc * Q[PH + r][PH + c];
    }
}

__global__ __launch_bounds__(NT) void split2_synthesis_kernel(SplitArgs A, Lift L) {
    __shared__ float Q[PN][PLD];
    int pp, tile, b, ctiles;
    pair_decode(A, xcd_remap(blockIdx.x, gridDim.x), pp, tile, b, ctiles);
    const SplitGeom g = split_geom(A, pp);
    const bool vertical = pp >= (1 << (A.t - 2));
    const int r0 = (tile / ctiles) * PT, k0 = (tile % ctiles) * PT;
    // `parent` holds the grandchildren (input), `child` the parent (output)
    const int64_t gsize = A.plane_elems >> (A.t + 1);
    const float* in = A.parent + b * A.parent_plane;
    for (int idx = threadIdx.x; idx < PN * PN; idx += NT) {
        const int r = idx / PN, c = idx - r * PN;
        const int i = r0 - PH + r, k = k0 - PH + c;
        const int ii = wrap(i, g.nr);
        const int pos = grandchild_pos(vertical, pp, ii & 3);
        const float sc = A.use_scale ? A.scale[pos] : 1.f;
        Q[r][c] = sc * in[pos * gsize + int64_t(ii >> 2) * g.nc + wrap(k - g.a * i, g.nc)];
    }
    __syncthreads();
    for (int s = 0; s < 4; ++s) {
        step_pair_second(Q, (L.first_odd + s) & 1, 0.5f * L.c[s], 2 + 2 * s);
        __syncthreads();
    }
    for (int s = 0; s < 4; ++s) {
        step_pair_first(Q, (L.first_odd + s) & 1, 0.5f * L.c[s], 9 + s);
        __syncthreads();
    }
    float* P = A.child + b * A.child_plane + g.parent_off;
    for (int idx = threadIdx.x; idx < PT * PT; idx += NT) {
        const int r = idx / PT, c = idx - r * PT;
        const int i = r0 + r, k = k0 + c;
        if (i >= g.nr || k >= g.nc) continue;
        P[int64_t(i) * g.nc + wrap(k - g.a * i, g.nc)] = Q[PH + r][PH + c];
    }
}

}  // namespace

hipError_t launch_dfb12_analysis(CView d, int R, int C, Quad out, Lift lift, int batch,
                                 hipStream_t st) {
    dim3 grid(((C + QT - 1) / QT) * ((R + QT - 1) / QT) * batch);
    dfb12_analysis_kernel<<<grid, NT, 0, st>>>(d, R, C, out, lift);
    return hipGetLastError();
}

hipError_t launch_dfb12_synthesis(Quad in, int R, int C, View d, Lift lift, int batch,
                                  hipStream_t st) {
    dim3 grid(((C + QT - 1) / QT) * ((R + QT - 1) / QT) * batch);
    dfb12_synthesis_kernel<<<grid, NT, 0, st>>>(in, R, C, d, lift);
    return hipGetLastError();
}

static int split_blocks(const SplitArgs& a, int batch) {
    // horizontal parents: (Rj >> (t-2)) x (Cj/2); vertical: (Cj >> (t-2)) x (Rj/2)
    const int t = a.t;
    auto tiles = [](int nr, int nc) { return ((nr + ST_R - 1) / ST_R) * ((nc + ST_C - 1) / ST_C); };
    const int th = tiles(a.Rj >> (t - 2), a.Cj >> 1);
    const int tv = tiles(a.Cj >> (t - 2), a.Rj >> 1);
    return (1 << (t - 2)) * (th + tv) * batch;
}

hipError_t launch_dfb_split_analysis(const SplitArgs& a, Lift lift, int batch, hipStream_t st) {
    dim3 grid(split_blocks(a, batch));
    split_analysis_kernel<<<grid, NT, 0, st>>>(a, lift);
    return hipGetLastError();
}

hipError_t launch_dfb_split_synthesis(const SplitArgs& a, Lift lift, int batch, hipStream_t st) {
    dim3 grid(split_blocks(a, batch));
    split_synthesis_kernel<<<grid, NT, 0, st>>>(a, lift);
    return hipGetLastError();
}

static int pair_blocks(const SplitArgs& a, int batch) {
    const int t = a.t;
    auto tiles = [](int nr, int nc) { return ((nr + PT - 1) / PT) * ((nc + PT - 1) / PT); };
    const int th = tiles(a.Rj >> (t - 2), a.Cj >> 1);
    const int tv = tiles(a.Cj >> (t - 2), a.Rj >> 1);
    return (1 << (t - 2)) * (th + tv) * batch;
}

hipError_t launch_dfb_split2_analysis(const SplitArgs& a, Lift lift, int batch, hipStream_t st) {
    split2_analysis_kernel<<<dim3(pair_blocks(a, batch)), NT, 0, st>>>(a, lift);
    return hipGetLastError();
}

hipError_t launch_dfb_split2_synthesis(const SplitArgs& a, Lift lift, int batch, hipStream_t st) {
    split2_synthesis_kernel<<<dim3(pair_blocks(a, batch)), NT, 0, st>>>(a, lift);
    return hipGetLastError();
}

}  // namespace ct

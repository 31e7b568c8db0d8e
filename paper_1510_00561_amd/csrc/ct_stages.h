// Tile stages of the contourlet pipeline, written once and used both by the
// per-stage persistent kernels and by the batched work-queue kernel.
//
// Every stage processes independent tiles and exposes
//   tiles()                    number of tiles,
//   fetch(tile, regs)          issue the tile's global loads into registers,
//   stage(tile, regs, smem)    write those registers into LDS,
//   compute(tile, smem)        the rest (LDS work and global stores).
// tile_loop() runs a stage over an XCD-contiguous range of tiles and fetches
// tile n+1 while tile n computes, so global-load latency hides behind LDS
// work even at two workgroups per CU.
#pragma once

#include "ct_device.h"

namespace ct {
namespace stage {

using namespace dev;

// ================================================================ driver
template <class S>
__device__ __forceinline__ void tile_range(int total, int& t0, int& t1, int& stride, int& first) {
    const int nwg = gridDim.x;
    const int x = blockIdx.x % kNumXcd, slot = blockIdx.x / kNumXcd;
    const int wbase = nwg / kNumXcd, wrem = nwg % kNumXcd;
    stride = wbase + (x < wrem ? 1 : 0);               // workgroups on this XCD
    const int tb = total / kNumXcd, tr = total % kNumXcd;
    t0 = x * tb + (x < tr ? x : tr);
    t1 = t0 + tb + (x < tr ? 1 : 0);
    first = t0 + slot;
}

template <class S>
__device__ __forceinline__ void tile_loop(S& st, float* smem) {
    int t0, t1, stride, t;
    tile_range<S>(st.tiles(), t0, t1, stride, t);
    typename S::Regs r;
    if (t < t1) st.fetch(t, r);
    while (t < t1) {
        const int tn = t + stride;
        st.stage(t, r, smem);
        __syncthreads();
        if (tn < t1) st.fetch(tn, r);
        st.compute(t, smem);
        __syncthreads();
        t = tn;
    }
}

// One tile with no prefetch (work-queue use): loads go straight to LDS,
// so no register staging array is live.
template <class S>
__device__ __forceinline__ void run_one(S& st, int tile, float* smem) {
    st.load_direct(tile, smem);
    __syncthreads();
    st.compute(tile, smem);
    __syncthreads();
}

// ================================================================ level analysis
// LP level + DFB tree levels 1-2, 64 x 64 tiles of the level image, 16-pixel halo.
struct LevelAnaArgs {
    CView src;
    int src_h, src_w, pad_mode;
    int R, C;
    View c_out;
    Quad out;
    Taps5 lo, up;
    Lift L;
    int batch;
};

template <int LO_R, int UP_R, int NT>
struct LevelAna {
    static constexpr int TO = 64, HD = 8, HL = 8;
    static constexpr int IN = TO + 2 * HD + 2 * HL;   // 96
    static constexpr int LD = IN + 1;
    static constexpr int D = TO + 2 * HD;             // 80
    static constexpr int CN = D / 2 + 4;              // 44
    static constexpr int CLD = CN + 1;
    static constexpr int UHLD = D + 1;
    static constexpr int HF_N = IN * CLD, UH_N = CN * UHLD;
    static constexpr int UNION_N = HF_N > UH_N ? HF_N : UH_N;
    static constexpr int SMEM = IN * LD + UNION_N + CN * CLD;   // floats
    static constexpr int NLOAD = (IN * IN + NT - 1) / NT;
    struct Regs {
        float v[NLOAD];
    };
    const LevelAnaArgs& A;
    int gx, gy;
    float invR, invC;
    __device__ LevelAna(const LevelAnaArgs& a) : A(a) {
        gx = (a.C + TO - 1) / TO;
        gy = (a.R + TO - 1) / TO;
        invR = 1.f / float(a.R);
        invC = 1.f / float(a.C);
    }
    __device__ int tiles() const { return gx * gy * A.batch; }
    __device__ void coords(int tile, int& n0, int& m0, int& b) const {
        m0 = (tile % gx) * TO;
        n0 = ((tile / gx) % gy) * TO;
        b = tile / (gx * gy);
    }
    // input sample at tile-local (rr, cc), periodic, padded past the frame
    __device__ float value(const float* sp, int n0, int m0, int rr, int cc) const {
        constexpr int H0 = HD + HL;
        int gr = fwrap(n0 - H0 + rr, A.R, invR), gc = fwrap(m0 - H0 + cc, A.C, invC);
        if (A.pad_mode == kPadReflect) {
            if (gr >= A.src_h) gr = 2 * A.src_h - 1 - gr;
            if (gc >= A.src_w) gc = 2 * A.src_w - 1 - gc;
        } else if (A.pad_mode == kPadZero) {
            if (gr >= A.src_h || gc >= A.src_w) return 0.f;
        }
        return sp[int64_t(gr) * A.src.ld + gc];
    }
    __device__ void fetch(int tile, Regs& r) const {
        int n0, m0, b;
        coords(tile, n0, m0, b);
        const float* sp = A.src.p + b * A.src.plane;
#pragma unroll
        for (int k = 0; k < NLOAD; ++k) {
            const int idx = threadIdx.x + k * NT;
            if (idx < IN * IN) {
                const int rr = idx / IN, cc = idx - rr * IN;
                r.v[k] = value(sp, n0, m0, rr, cc);
            }
        }
    }
    __device__ void load_direct(int tile, float* smem) const {
        int n0, m0, b;
        coords(tile, n0, m0, b);
        const float* sp = A.src.p + b * A.src.plane;
        for (int idx = threadIdx.x; idx < IN * IN; idx += NT) {
            const int rr = idx / IN, cc = idx - rr * IN;
            smem[rr * LD + cc] = value(sp, n0, m0, rr, cc);
        }
    }
    __device__ void stage(int, const Regs& r, float* smem) const {
#pragma unroll
        for (int k = 0; k < NLOAD; ++k) {
            const int idx = threadIdx.x + k * NT;
            if (idx < IN * IN) {
                const int rr = idx / IN, cc = idx - rr * IN;
                smem[rr * LD + cc] = r.v[k];
            }
        }
    }
    __device__ void compute(int tile, float* smem) const {
        int n0, m0, b;
        coords(tile, n0, m0, b);
        float* in = smem;
        float* hf = smem + IN * LD;
        float* uh = hf;
        float* c = hf + UNION_N;
        rows_lo<LO_R, IN, CN, LD, CLD, NT>(in, hf, A.lo);
        __syncthreads();
        const int Rh = A.R >> 1, Ch = A.C >> 1;
        float* cp = A.c_out.p + b * A.c_out.plane;
        constexpr int OFF = (HD + 4) / 2;   // first owned lowpass sample
        for (int idx = threadIdx.x; idx < CN * CN; idx += NT) {
            const int ss = idx / CN, t = idx - ss * CN;
            const float v = cols_lo<LO_R, CLD>(hf, A.lo, ss, t);
            c[ss * CLD + t] = v;
            if (ss >= OFF && ss < OFF + TO / 2 && t >= OFF && t < OFF + TO / 2) {
                const int gr = (n0 >> 1) + ss - OFF, gc = (m0 >> 1) + t - OFF;
                if (gr < Rh && gc < Ch) cp[int64_t(gr) * A.c_out.ld + gc] = v;
            }
        }
        __syncthreads();
        rows_up<UP_R, CN, D, CLD, UHLD, NT>(c, uh, A.up);
        __syncthreads();
        float* T = in + HL * LD + HL;
        for (int idx = threadIdx.x; idx < D * D; idx += NT) {
            const int i = idx / D, j = idx - i * D;
            T[i * LD + j] -= cols_up<UP_R, UHLD>(uh, A.up, i, j);
        }
        __syncthreads();
        int m = 1;
        for (int st = 0; st < 4; ++st, ++m) {
            step_cross<D, LD, NT>(T, (A.L.first_odd + st) & 1, 0.5f * A.L.c[st], m);
            __syncthreads();
        }
        for (int st = 0; st < 4; ++st, ++m) {
            step_diag<D, LD, NT>(T, (A.L.first_odd + st) & 1, 0.5f * A.L.c[st], m);
            __syncthreads();
        }
        constexpr int HQ = TO / 2;
        for (int idx = threadIdx.x; idx < 2 * HQ * HQ; idx += NT) {
            const int q = idx / (HQ * HQ);
            const int rem = idx - q * HQ * HQ;
            const int i = rem / HQ, k = rem - i * HQ;
            const int pr = q == 0 ? 0 : 1, pc = q == 0 ? 1 : 0;
            const int gi = (n0 >> 1) + i, gk = (m0 >> 1) + k;
            if (gi < Rh && gk < Ch)
                A.out.p[q][b * A.out.plane + int64_t(gi) * Ch + gk] =
                    A.out.scale[q] * T[(HD + 2 * i + pr) * LD + HD + 2 * k + pc];
        }
        for (int idx = threadIdx.x; idx < 2 * HQ * HQ; idx += NT) {
            const int q = 2 + idx / (HQ * HQ);
            const int rem = idx - (q - 2) * HQ * HQ;
            const int k = rem / HQ, i = rem - k * HQ;
            const int p = q == 2 ? 0 : 1;
            const int gi = (n0 >> 1) + i, gk = (m0 >> 1) + k;
            if (gi < Rh && gk < Ch)
                A.out.p[q][b * A.out.plane + int64_t(gk) * Rh + gi] =
                    A.out.scale[q] * T[(HD + 2 * i + p) * LD + HD + 2 * k + p];
        }
    }
};

// ================================================================ level synthesis
// DFB tree levels 1-2 back to the bandpass image, then dual LP synthesis.
struct LevelSynArgs {
    Quad in;
    CView c_in;
    int R, C;
    View x_out;
    int out_h, out_w;
    Taps5 lo, up;
    Lift L;
    int batch;
};

template <int LO_R, int UP_R, int NT>
struct LevelSyn {
    static constexpr int TO = 64, HD = 8, HL = 8;
    static constexpr int T = TO + 2 * HL + 2 * HD;    // 96
    static constexpr int LD = T + 1;
    static constexpr int D = TO + 2 * HL;             // 80
    static constexpr int CN = TO / 2 + 4;             // 36
    static constexpr int CLD = CN + 1;
    static constexpr int UHLD = TO + 1;
    static constexpr int HF_N = D * CLD, UH_N = CN * UHLD;
    static constexpr int UNION_N = HF_N > UH_N ? HF_N : UH_N;
    static constexpr int SMEM = T * LD + UNION_N + CN * CLD;
    static constexpr int HN = T / 2;                  // 48 compact samples per axis
    static constexpr int NQ = 2 * HN * HN;            // per cone pair
    static constexpr int NTOT = 2 * NQ + CN * CN;
    static constexpr int NLOAD = (NTOT + NT - 1) / NT;
    struct Regs {
        float v[NLOAD];
    };
    const LevelSynArgs& A;
    int gx, gy;
    float invRh, invCh;
    __device__ LevelSyn(const LevelSynArgs& a) : A(a) {
        gx = (a.C + TO - 1) / TO;
        gy = (a.R + TO - 1) / TO;
        invRh = 1.f / float(a.R >> 1);
        invCh = 1.f / float(a.C >> 1);
    }
    __device__ int tiles() const { return gx * gy * A.batch; }
    __device__ void coords(int tile, int& n0, int& m0, int& b) const {
        m0 = (tile % gx) * TO;
        n0 = ((tile / gx) % gy) * TO;
        b = tile / (gx * gy);
    }
    // slot idx -> (global pointer or LDS index); horizontal channels run
    // along compact columns, vertical ones (transposed) along compact rows
    __device__ void locate(int idx, int n0, int m0, int b, const float*& src, float& sc,
                           int& lds) const {
        const int Rh = A.R >> 1, Ch = A.C >> 1;
        constexpr int H0 = (HD + HL) / 2;
        if (idx < NQ) {
            const int q = idx / (HN * HN);
            const int rem = idx - q * HN * HN;
            const int i = rem / HN, k = rem - i * HN;
            const int pr = q == 0 ? 0 : 1, pc = q == 0 ? 1 : 0;
            const int gi = fwrap((n0 >> 1) - H0 + i, Rh, invRh), gk = fwrap((m0 >> 1) - H0 + k, Ch, invCh);
            src = A.in.p[q] + b * A.in.plane + int64_t(gi) * Ch + gk;
            sc = A.in.scale[q];
            lds = (2 * i + pr) * LD + 2 * k + pc;
        } else if (idx < 2 * NQ) {
            const int j = idx - NQ;
            const int q = 2 + j / (HN * HN);
            const int rem = j - (q - 2) * HN * HN;
            const int k = rem / HN, i = rem - k * HN;
            const int p = q == 2 ? 0 : 1;
            const int gi = fwrap((n0 >> 1) - H0 + i, Rh, invRh), gk = fwrap((m0 >> 1) - H0 + k, Ch, invCh);
            src = A.in.p[q] + b * A.in.plane + int64_t(gk) * Rh + gi;
            sc = A.in.scale[q];
            lds = (2 * i + p) * LD + 2 * k + p;
        } else {
            const int j = idx - 2 * NQ;
            const int ss = j / CN, t = j - ss * CN;
            const int gr = fwrap((n0 >> 1) - 2 + ss, Rh, invRh), gc = fwrap((m0 >> 1) - 2 + t, Ch, invCh);
            src = A.c_in.p + b * A.c_in.plane + int64_t(gr) * A.c_in.ld + gc;
            sc = 1.f;
            lds = T * LD + UNION_N + ss * CLD + t;    // the lowpass tile
        }
    }
    __device__ void fetch(int tile, Regs& r) const {
        int n0, m0, b;
        coords(tile, n0, m0, b);
#pragma unroll
        for (int k = 0; k < NLOAD; ++k) {
            const int idx = threadIdx.x + k * NT;
            if (idx < NTOT) {
                const float* src;
                float sc;
                int lds;
                locate(idx, n0, m0, b, src, sc, lds);
                r.v[k] = sc * *src;
            }
        }
    }
    __device__ void stage(int tile, const Regs& r, float* smem) const {
        int n0, m0, b;
        coords(tile, n0, m0, b);
#pragma unroll
        for (int k = 0; k < NLOAD; ++k) {
            const int idx = threadIdx.x + k * NT;
            if (idx < NTOT) {
                const float* src;
                float sc;
                int lds;
                locate(idx, n0, m0, b, src, sc, lds);
                smem[lds] = r.v[k];
            }
        }
    }
    __device__ void load_direct(int tile, float* smem) const {
        int n0, m0, b;
        coords(tile, n0, m0, b);
        for (int idx = threadIdx.x; idx < NTOT; idx += NT) {
            const float* src;
            float sc;
            int lds;
            locate(idx, n0, m0, b, src, sc, lds);
            smem[lds] = sc * *src;
        }
    }
    __device__ void compute(int tile, float* smem) const {
        int n0, m0, b;
        coords(tile, n0, m0, b);
        float* t = smem;
        float* hf = smem + T * LD;
        float* uh = hf;
        float* c = hf + UNION_N;
        int m = 1;
        for (int st = 0; st < 4; ++st, ++m) {
            step_diag<T, LD, NT>(t, (A.L.first_odd + st) & 1, 0.5f * A.L.c[st], m);
            __syncthreads();
        }
        for (int st = 0; st < 4; ++st, ++m) {
            step_cross<T, LD, NT>(t, (A.L.first_odd + st) & 1, 0.5f * A.L.c[st], m);
            __syncthreads();
        }
        const float* Dp = t + HD * LD + HD;
        rows_lo<LO_R, D, CN, LD, CLD, NT>(Dp, hf, A.lo);
        __syncthreads();
        for (int idx = threadIdx.x; idx < CN * CN; idx += NT) {
            const int ss = idx / CN, tt = idx - ss * CN;
            c[ss * CLD + tt] -= cols_lo<LO_R, CLD>(hf, A.lo, ss, tt);
        }
        __syncthreads();
        rows_up<UP_R, CN, TO, CLD, UHLD, NT>(c, uh, A.up);
        __syncthreads();
        float* xp = A.x_out.p + b * A.x_out.plane;
        for (int idx = threadIdx.x; idx < TO * TO; idx += NT) {
            const int i = idx / TO, j = idx - i * TO;
            const int gr = n0 + i, gc = m0 + j;
            if (gr < A.R && gc < A.C && gr < A.out_h && gc < A.out_w)
                xp[int64_t(gr) * A.x_out.ld + gc] =
                    Dp[(HL + i) * LD + HL + j] + cols_up<UP_R, UHLD>(uh, A.up, i, j);
        }
    }
};

// ================================================================ DFB splits
// Geometry of a parent channel at tree level t-1 (split at level t).
struct SplitGeom {
    int nr, nc;             // parent array size (vertical channels transposed)
    float inv_nr, inv_nc;
    int a;                  // shear parameter
    bool vertical;
    int64_t parent_off;     // parent channel offset within a plane
    int even_pos, odd_pos;  // child channel positions at level t
};

__device__ __forceinline__ SplitGeom split_geom(const SplitArgs& A, int pp) {
    SplitGeom g;
    const int t = A.t;
    const int hp = 1 << (t - 2);                 // horizontal parents
    g.vertical = pp >= hp;
    const int q = 1 << (t - 3);
    if (!g.vertical) {
        g.a = pp - q;
        g.nr = A.Rj >> (t - 2);
        g.nc = A.Cj >> 1;
        g.odd_pos = 2 * pp;          // a' = 2a
        g.even_pos = 2 * pp + 1;     // a' = 2a + 1
    } else {
        g.a = q - 1 - (pp - hp);
        g.nr = A.Cj >> (t - 2);
        g.nc = A.Rj >> 1;
        g.even_pos = 2 * pp;
        g.odd_pos = 2 * pp + 1;
    }
    g.parent_off = pp * (A.plane_elems >> (t - 1));
    g.inv_nr = 1.f / float(g.nr);
    g.inv_nc = 1.f / float(g.nc);
    return g;
}

// Logical tile -> (parent channel, tile within it, plane): per plane the
// horizontal parents come first, each with th tiles, then the vertical ones.
template <int TR, int TC>
__device__ __forceinline__ void split_decode(const SplitArgs& A, int L, int& pp, int& rt, int& ct,
                                             int& b) {
    const int t = A.t;
    const int cth = ((A.Cj >> 1) + TC - 1) / TC, ctv = ((A.Rj >> 1) + TC - 1) / TC;
    const int th = (((A.Rj >> (t - 2)) + TR - 1) / TR) * cth;
    const int tv = (((A.Cj >> (t - 2)) + TR - 1) / TR) * ctv;
    const int nh = 1 << (t - 2);
    const int per_plane = nh * (th + tv);
    b = L / per_plane;
    int rem = L - b * per_plane;
    int tile, ctiles;
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
    rt = tile / ctiles;
    ct = tile - rt * ctiles;
}

template <int TR, int TC>
__device__ __forceinline__ int split_tiles(const SplitArgs& A, int batch) {
    const int t = A.t;
    const int th = (((A.Rj >> (t - 2)) + TR - 1) / TR) * (((A.Cj >> 1) + TC - 1) / TC);
    const int tv = (((A.Cj >> (t - 2)) + TR - 1) / TR) * (((A.Rj >> 1) + TC - 1) / TC);
    return (1 << (t - 2)) * (th + tv) * batch;
}

// Channel position of grandchild class (row i & 3) of parent pp at level t+1.
__device__ __forceinline__ int grandchild_pos(bool vertical, int pp, int cls) {
    // horizontal: even child 2pp+1 (children 4pp+3, 4pp+2), odd child 2pp (4pp+1, 4pp)
    // vertical:   even child 2pp   (children 4pp, 4pp+1),   odd child 2pp+1 (4pp+2, 4pp+3)
    const int h = (cls & 1) ? 1 - (cls >> 1) : 3 - (cls >> 1);
    const int v = ((cls & 1) << 1) | (cls >> 1);
    return 4 * pp + (vertical ? v : h);
}

// One tree level (LEVELS == 1, 32 x 64 tiles, halo 4) or two consecutive
// tree levels (LEVELS == 2, 64 x 64 tiles, halo 12), analysis (ANA) or
// synthesis, in the sheared frame Q[i, k] = P[i, k - a i] of the parent.
// Level t:   N = Q[i-1][k+1] + Q[i+1][k-1] - Q[i-1][k] - Q[i+1][k]
// Level t+1: even rows  N = Q[i-2][k+2] + Q[i+2][k-2] - Q[i-2][k+1] - Q[i+2][k-1]
//            odd rows   N = Q[i-2][k+1] + Q[i+2][k-1] - Q[i-2][k]   - Q[i+2][k]
// (all halved; sub-parity of row i at level t+1 is (i >> 1) & 1).
template <int LEVELS, bool ANA, int NT>
struct Split {
    static constexpr int TR = LEVELS == 1 ? 32 : 64;
    static constexpr int TC = 64;
    static constexpr int H = LEVELS == 1 ? 4 : 12;
    static constexpr int NR = TR + 2 * H, NC = TC + 2 * H;
    static constexpr int LD = NC + 1;
    static constexpr int SMEM = NR * LD;
    static constexpr int NLOAD = (NR * NC + NT - 1) / NT;
    struct Regs {
        float v[NLOAD];
    };
    const SplitArgs& A;
    int batch;
    Lift lift;
    __device__ Split(const SplitArgs& a, int b, const Lift& L) : A(a), batch(b), lift(L) {}
    __device__ int tiles() const { return split_tiles<TR, TC>(A, batch); }

    // input sample for sheared position (i unwrapped, k) of parent pp
    __device__ float load(const SplitGeom& g, int pp, int b, int i, int k) const {
        const int col = fwrap(k - g.a * i, g.nc, g.inv_nc);
        if (ANA) {
            const float* P = A.parent + b * A.parent_plane + g.parent_off;
            return P[int64_t(fwrap(i, g.nr, g.inv_nr)) * g.nc + col];
        }
        const int ii = fwrap(i, g.nr, g.inv_nr);
        const float* in = A.parent + b * A.parent_plane;
        if (LEVELS == 1) {
            const int64_t cs = A.plane_elems >> A.t;
            const int pos = (ii & 1) ? g.odd_pos : g.even_pos;
            const float sc = A.use_scale ? A.scale[pos] : 1.f;
            return sc * in[pos * cs + int64_t(ii >> 1) * g.nc + col];
        }
        const int64_t gs = A.plane_elems >> (A.t + 1);
        const int pos = grandchild_pos(g.vertical, pp, ii & 3);
        const float sc = A.use_scale ? A.scale[pos] : 1.f;
        return sc * in[pos * gs + int64_t(ii >> 2) * g.nc + col];
    }
    __device__ void fetch(int tile, Regs& r) const {
        int pp, rt, ct, b;
        split_decode<TR, TC>(A, tile, pp, rt, ct, b);
        const SplitGeom g = split_geom(A, pp);
        const int r0 = rt * TR, k0 = ct * TC;
#pragma unroll
        for (int j = 0; j < NLOAD; ++j) {
            const int idx = threadIdx.x + j * NT;
            if (idx < NR * NC) {
                const int rr = idx / NC, cc = idx - rr * NC;
                r.v[j] = load(g, pp, b, r0 - H + rr, k0 - H + cc);
            }
        }
    }
    __device__ void stage(int, const Regs& r, float* smem) const {
#pragma unroll
        for (int j = 0; j < NLOAD; ++j) {
            const int idx = threadIdx.x + j * NT;
            if (idx < NR * NC) {
                const int rr = idx / NC, cc = idx - rr * NC;
                smem[rr * LD + cc] = r.v[j];
            }
        }
    }
    __device__ void load_direct(int tile, float* smem) const {
        int pp, rt, ct, b;
        split_decode<TR, TC>(A, tile, pp, rt, ct, b);
        const SplitGeom g = split_geom(A, pp);
        const int r0 = rt * TR, k0 = ct * TC;
        for (int idx = threadIdx.x; idx < NR * NC; idx += NT) {
            const int rr = idx / NC, cc = idx - rr * NC;
            smem[rr * LD + cc] = load(g, pp, b, r0 - H + rr, k0 - H + cc);
        }
    }
    // level-t step on rows of parity par over rows [m, NR - m), cols [m, NC - m)
    __device__ void step1(float* Q, int par, float coef, int m) const {
        const int rows = (NR - 2 * m) / 2, cols = NC - 2 * m;
        const int first = m + ((m + par) & 1);
        const int q = NT / cols, rmd = NT - q * cols;
        int rr = threadIdx.x / cols, cc = threadIdx.x - rr * cols;
        while (rr < rows) {
            float* p = Q + (first + 2 * rr) * LD + m + cc;
            *p += coef * ((p[-LD + 1] + p[LD - 1]) - (p[-LD] + p[LD]));
            rr += q;
            cc += rmd;
            if (cc >= cols) {
                cc -= cols;
                ++rr;
            }
        }
    }
    // level-(t+1) step on rows with (r >> 1) & 1 == par; m even
    __device__ void step2(float* Q, int par, float coef, int m) const {
        const int rows = (NR - 2 * m) / 2, cols = NC - 2 * m;
        const int first = m + ((((m >> 1) & 1) == par) ? 0 : 2);
        const int q = NT / cols, rmd = NT - q * cols;
        int rr = threadIdx.x / cols, cc = threadIdx.x - rr * cols;
        while (rr < rows) {
            const int r = first + 4 * (rr >> 1) + (rr & 1);
            const int e = (~r) & 1;   // even rows: the even child's extra shift
            float* p = Q + r * LD + m + cc;
            *p += coef * ((p[-2 * LD + 1 + e] + p[2 * LD - 1 - e]) - (p[-2 * LD + e] + p[2 * LD - e]));
            rr += q;
            cc += rmd;
            if (cc >= cols) {
                cc -= cols;
                ++rr;
            }
        }
    }
    __device__ void compute(int tile, float* Q) const {
        int pp, rt, ct, b;
        split_decode<TR, TC>(A, tile, pp, rt, ct, b);
        const SplitGeom g = split_geom(A, pp);
        const int r0 = rt * TR, k0 = ct * TC;
        const Lift& L = lift;
        if (ANA) {
            for (int s = 0; s < 4; ++s) {
                step1(Q, (L.first_odd + s) & 1, 0.5f * L.c[s], s + 1);
                __syncthreads();
            }
            if (LEVELS == 2) {
                for (int s = 0; s < 4; ++s) {
                    step2(Q, (L.first_odd + s) & 1, 0.5f * L.c[s], 6 + 2 * s);
                    __syncthreads();
                }
            }
            float* out = A.child + b * A.child_plane;
            for (int idx = threadIdx.x; idx < TR * TC; idx += NT) {
                const int rr = idx / TC, cc = idx - rr * TC;
                const int i = r0 + rr, k = k0 + cc;
                if (i >= g.nr || k >= g.nc) continue;
                const int col = fwrap(k - g.a * i, g.nc, g.inv_nc);
                const float v = Q[(H + rr) * LD + H + cc];
                if (LEVELS == 1) {
                    const int pos = (i & 1) ? g.odd_pos : g.even_pos;
                    const float sc = A.use_scale ? A.scale[pos] : 1.f;
                    out[pos * (A.plane_elems >> A.t) + int64_t(i >> 1) * g.nc + col] = sc * v;
                } else {
                    const int pos = grandchild_pos(g.vertical, pp, i & 3);
                    const float sc = A.use_scale ? A.scale[pos] : 1.f;
                    out[pos * (A.plane_elems >> (A.t + 1)) + int64_t(i >> 2) * g.nc + col] = sc * v;
                }
            }
        } else {
            if (LEVELS == 2) {
                for (int s = 0; s < 4; ++s) {
                    step2(Q, (L.first_odd + s) & 1, 0.5f * L.c[s], 2 + 2 * s);
                    __syncthreads();
                }
            }
            const int mb = LEVELS == 2 ? 9 : 1;
            for (int s = 0; s < 4; ++s) {
                step1(Q, (L.first_odd + s) & 1, 0.5f * L.c[s], mb + s);
                __syncthreads();
            }
            float* P = A.child + b * A.child_plane + g.parent_off;
            for (int idx = threadIdx.x; idx < TR * TC; idx += NT) {
                const int rr = idx / TC, cc = idx - rr * TC;
                const int i = r0 + rr, k = k0 + cc;
                if (i >= g.nr || k >= g.nc) continue;
                P[int64_t(i) * g.nc + fwrap(k - g.a * i, g.nc, g.inv_nc)] = Q[(H + rr) * LD + H + cc];
            }
        }
    }
};

}  // namespace stage
}  // namespace ct

// Filters and lifting constants of the 9-7 pair and of the LeGall 5/3 variant
// (host only, double precision).
//
// Paper section 2.1: LP and DFB use the Cohen-Daubechies 9-7 biorthogonal
// filters. Construction used here:
//   y = (1 - t)/2 with t = cos(w); Q(y) = 1 + 4y + 10y^2 + 20y^3 has a real
//   root y_r and a complex pair. Writing Q(y) = (y - y_r) Q2(y),
//     analysis lowpass  p(t) ~ ((1+t)/2)^2 Q2((1-t)/2)    (9 taps)
//     synthesis lowpass q(t) ~ ((1+t)/2)^2 ((1-t)/2 - y_r) (7 taps)
//   each normalised to sqrt(2) at t = 1, then expanded into taps with
//   t^k = ((z + 1/z)/2)^k.
// LP filters are hbar = h / sqrt(2) (sum 1) and gbar = g * sqrt(2) (sum 2).
//
// Lifting: the fan filter bank runs as four lifting steps plus a scaling,
// the Daubechies-Sweldens factorisation of the same pair. Its constants are
// refined here by Newton's method from their published 10-digit values until
// the lifted analysis lowpass reproduces the closed-form taps to rounding,
// and the lifted highpass is then checked against q(-t).
//
// Variant: the LeGall 5/3 pair, the same construction with two zeros at
// w = pi on each side: Q(y) = 1 + 2y goes whole to the analysis side,
//     p(t) ~ ((1+t)/2)(1 + (1-t))    (5 taps),   q(t) ~ (1+t)/2   (3 taps).
// Its lifting is two steps, predict -1/2 and update 1/4, with the scaling
// sqrt 2; the same two checks confirm them.
#include <math.h>
#include <string.h>

#include <mutex>

#include "ct_internal.h"

namespace ct {
namespace {

// Polynomial helpers (coefficients lowest degree first).
struct Poly {
    double c[8];
    int n;  // number of coefficients
};

Poly pmul(const Poly& a, const Poly& b) {
    Poly r;
    memset(&r, 0, sizeof(r));
    r.n = a.n + b.n - 1;
    for (int i = 0; i < a.n; ++i)
        for (int j = 0; j < b.n; ++j) r.c[i + j] += a.c[i] * b.c[j];
    return r;
}

double peval(const Poly& a, double x) {
    double y = 0;
    for (int i = a.n - 1; i >= 0; --i) y = y * x + a.c[i];
    return y;
}

// taps[0..deg] of the symmetric Laurent polynomial P((z + 1/z)/2):
// out[k] is the coefficient of z^k (= of z^-k).
void chebyshev_taps(const Poly& p, double* out) {
    const int deg = p.n - 1;
    const int W = 2 * deg + 1;
    double acc[32], pw[32], nx[32];
    memset(acc, 0, sizeof(acc));
    memset(pw, 0, sizeof(pw));
    pw[deg] = 1.0;
    for (int k = 0; k < p.n; ++k) {
        for (int i = 0; i < W; ++i) acc[i] += p.c[k] * pw[i];
        memset(nx, 0, sizeof(nx));
        for (int i = 0; i < W; ++i) {
            if (i + 1 < W) nx[i + 1] += 0.5 * pw[i];
            if (i - 1 >= 0) nx[i - 1] += 0.5 * pw[i];
        }
        memcpy(pw, nx, sizeof(pw));
    }
    for (int k = 0; k <= deg; ++k) out[k] = acc[deg + k];
}

// One 1-D analysis by lifting on a torus of length N; x is overwritten.
void lift1d(double* x, int N, const double* th) {
    const double al = th[0], be = th[1], ga = th[2], de = th[3], ze = th[4];
    auto at = [&](int i) -> double& { return x[((i % N) + N) % N]; };
    for (int i = 1; i < N; i += 2) at(i) += al * (at(i - 1) + at(i + 1));
    for (int i = 0; i < N; i += 2) at(i) += be * (at(i - 1) + at(i + 1));
    for (int i = 1; i < N; i += 2) at(i) += ga * (at(i - 1) + at(i + 1));
    for (int i = 0; i < N; i += 2) at(i) += de * (at(i - 1) + at(i + 1));
    for (int i = 0; i < N; ++i) x[i] *= (i % 2 == 0) ? ze : 1.0 / ze;
}

// Lifted lowpass taps h[0..4] (unit-energy normalisation, sum sqrt 2).
void lifted_lowpass(const double* th, double* h) {
    const int N = 32;
    double x[N];
    // impulse at 0: even outputs at 0, 2, 4 carry h[0], h[2], h[4]
    memset(x, 0, sizeof(x));
    x[0] = 1;
    lift1d(x, N, th);
    h[0] = x[0];
    h[2] = x[2];
    h[4] = x[4];
    // impulse at 1: even outputs at 0 (h[1]) and 4 (h[3])
    memset(x, 0, sizeof(x));
    x[1] = 1;
    lift1d(x, N, th);
    h[1] = x[0];
    h[3] = x[4];
}

bool solve5(double A[5][5], double* b) {
    for (int c = 0; c < 5; ++c) {
        int piv = c;
        for (int r = c + 1; r < 5; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (fabs(A[piv][c]) < 1e-300) return false;
        if (piv != c) {
            for (int k = 0; k < 5; ++k) {
                double t = A[c][k];
                A[c][k] = A[piv][k];
                A[piv][k] = t;
            }
            double t = b[c];
            b[c] = b[piv];
            b[piv] = t;
        }
        for (int r = c + 1; r < 5; ++r) {
            double f = A[r][c] / A[c][c];
            for (int k = c; k < 5; ++k) A[r][k] -= f * A[c][k];
            b[r] -= f * b[c];
        }
    }
    for (int c = 4; c >= 0; --c) {
        double s = b[c];
        for (int k = c + 1; k < 5; ++k) s -= A[c][k] * b[k];
        b[c] = s / A[c][c];
    }
    return true;
}

// Lowpass taps reproduced by the lifting th, and odd outputs equal to
// (-1)^n g[n] (the highpass q(-t)).
bool lifting_matches(const double* th, const double* h, const double* g) {
    double hl[5];
    lifted_lowpass(th, hl);
    bool ok = true;
    for (int i = 0; i < 5; ++i) ok = ok && fabs(hl[i] - h[i]) < 1e-12;
    const int N = 32;
    double x[N];
    for (int src = 0; src < 2; ++src) {
        memset(x, 0, sizeof(x));
        x[src] = 1;
        lift1d(x, N, th);
        for (int o = 1; o < N; o += 2) {
            int n = o - src;       // output at o sees tap gm[o - src]
            if (n > N / 2) n -= N;
            int an = n < 0 ? -n : n;
            double want = an <= 3 ? ((an % 2) ? -g[an] : g[an]) : 0.0;
            ok = ok && fabs(x[o] - want) < 1e-12;
        }
    }
    return ok;
}

Constants build53() {
    Constants k;
    memset(&k, 0, sizeof(k));
    Poly half_plus{{0.5, 0.5}, 2};
    Poly rem{{2.0, -1.0}, 2};              // 1 + 2y with y = (1 - t)/2
    Poly p = pmul(half_plus, rem);
    Poly q = half_plus;
    const double s2 = sqrt(2.0);
    const double np = s2 / peval(p, 1.0), nq = s2 / peval(q, 1.0);
    for (int i = 0; i < p.n; ++i) p.c[i] *= np;
    for (int i = 0; i < q.n; ++i) q.c[i] *= nq;
    double h[5] = {0, 0, 0, 0, 0}, g[4] = {0, 0, 0, 0};
    chebyshev_taps(p, h);
    chebyshev_taps(q, g);
    for (int i = 0; i < 5; ++i) k.hbar[i] = h[i] / s2;
    for (int i = 0; i < 4; ++i) k.gbar[i] = g[i] * s2;
    const double th[5] = {-0.5, 0.25, 0.0, 0.0, s2};
    k.alpha = th[0];
    k.beta = th[1];
    k.gamma = th[2];
    k.delta = th[3];
    k.zeta = th[4];
    k.ok = lifting_matches(th, h, g);
    return k;
}

Constants build97() {
    Constants k;
    memset(&k, 0, sizeof(k));
    // real root of 20y^3 + 10y^2 + 4y + 1 by Newton from -0.34
    double yr = -0.34;
    for (int it = 0; it < 60; ++it) {
        double f = ((20 * yr + 10) * yr + 4) * yr + 1;
        double df = (60 * yr + 20) * yr + 4;
        yr -= f / df;
    }
    // deflate: Q(y) = (y - yr)(20 y^2 + b y + c)
    const double qb = 10 + 20 * yr;
    const double qc = 4 + qb * yr;
    // substitute y = (1 - t)/2
    Poly half_plus{{0.5, 0.5}, 2};
    Poly cos4 = pmul(half_plus, half_plus);
    Poly y_of_t{{0.5, -0.5}, 2};
    Poly y2 = pmul(y_of_t, y_of_t);
    Poly quad;
    memset(&quad, 0, sizeof(quad));
    quad.n = 3;
    for (int i = 0; i < 3; ++i) quad.c[i] = 20 * y2.c[i] + (i < 2 ? qb * y_of_t.c[i] : 0.0);
    quad.c[0] += qc;
    Poly lin{{0.5 - yr, -0.5}, 2};
    Poly p = pmul(cos4, quad);
    Poly q = pmul(cos4, lin);
    const double s2 = sqrt(2.0);
    const double np = s2 / peval(p, 1.0), nq = s2 / peval(q, 1.0);
    for (int i = 0; i < p.n; ++i) p.c[i] *= np;
    for (int i = 0; i < q.n; ++i) q.c[i] *= nq;
    double h[5], g[4];
    chebyshev_taps(p, h);
    chebyshev_taps(q, g);
    for (int i = 0; i < 5; ++i) k.hbar[i] = h[i] / s2;
    for (int i = 0; i < 4; ++i) k.gbar[i] = g[i] * s2;

    // lifting constants: Newton on lifted_lowpass(theta) = h
    double th[5] = {-1.586134342, -0.05298011854, 0.8829110762, 0.4435068522, 1.149604398};
    for (int it = 0; it < 30; ++it) {
        double r[5];
        lifted_lowpass(th, r);
        double res[5], maxres = 0;
        for (int i = 0; i < 5; ++i) {
            res[i] = r[i] - h[i];
            maxres = fmax(maxres, fabs(res[i]));
        }
        if (maxres < 1e-15) break;
        double Jm[5][5];
        for (int c = 0; c < 5; ++c) {
            double tp[5], tm[5], rp[5], rm[5];
            memcpy(tp, th, sizeof(tp));
            memcpy(tm, th, sizeof(tm));
            const double step = 1e-6 * fmax(1.0, fabs(th[c]));
            tp[c] += step;
            tm[c] -= step;
            lifted_lowpass(tp, rp);
            lifted_lowpass(tm, rm);
            for (int i = 0; i < 5; ++i) Jm[i][c] = (rp[i] - rm[i]) / (2 * step);
        }
        if (!solve5(Jm, res)) break;
        for (int i = 0; i < 5; ++i) th[i] -= res[i];
    }
    k.alpha = th[0];
    k.beta = th[1];
    k.gamma = th[2];
    k.delta = th[3];
    k.zeta = th[4];
    k.ok = lifting_matches(th, h, g);
    return k;
}

}  // namespace

const Constants& constants(int filters) {
    static Constants k[2];
    static std::once_flag once;
    std::call_once(once, [] {
        k[CT_FILTERS_CDF97] = build97();
        k[CT_FILTERS_LEGALL53] = build53();
    });
    return k[filters == CT_FILTERS_LEGALL53 ? CT_FILTERS_LEGALL53 : CT_FILTERS_CDF97];
}

}  // namespace ct

// Host check of the quantiser's index functions (ct_quant_stages.h), built
// for the host only: quant_index(a, b, 1 / b) against to_index of the
// correctly rounded host division, for steps that stress the reciprocal
// (mantissas of all ones and near them, powers of two, the integers and
// halves, the ends of the fast range) and log-uniform steps, on values at
// and a few float32 steps around every (k + 1/2) b and on random values
// with quotients up to 2^26; and to_index against rounding halves away from
// zero written with floor on doubles, for random float bit patterns.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <random>
#include <vector>

#include "ct_quant_stages.h"

using ct::qstage::fast_step;
using ct::qstage::quant_index;
using ct::qstage::to_index;

static float bits_to_float(uint32_t u) {
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// round half away from zero, saturated to int16, NaN -> 0 (in double)
static int16_t ref_index(float v) {
    if (v != v) return 0;
    const double a = fabs(double(v)), r = copysign(floor(a + 0.5), double(v));
    if (r >= 32767.0) return 32767;
    if (r <= -32768.0) return -32768;
    return int16_t(r);
}

int main() {
    std::mt19937_64 g(2024);
    long long bad_round = 0, bad_q = 0, checked = 0;
    for (int i = 0; i < (1 << 24); ++i) {
        const float v = bits_to_float(uint32_t(g()));
        if (to_index(v) != ref_index(v)) {
            if (bad_round < 5) printf("to_index(%a) = %d, expected %d\n", v, to_index(v), ref_index(v));
            ++bad_round;
        }
    }
    // every float within 8 units in the last place of k + 1/2 (and of k)
    for (int k = -70000; k <= 70000; ++k) {
        for (float c : {float(k) + 0.5f, float(k)}) {
            float lo = c, hi = c;
            for (int u = 0; u < 8; ++u) {
                lo = nextafterf(lo, -INFINITY);
                hi = nextafterf(hi, INFINITY);
            }
            for (float v = lo; v <= hi; v = nextafterf(v, INFINITY)) {
                if (to_index(v) != ref_index(v)) {
                    if (bad_round < 5) printf("to_index(%a) = %d, expected %d\n", v, to_index(v), ref_index(v));
                    ++bad_round;
                }
            }
        }
    }
    std::vector<float> steps;
    for (int k = -20; k <= 19; ++k) {
        const float m[] = {2.f - ldexpf(1.f, -23), 2.f - ldexpf(1.f, -22), 1.f + ldexpf(1.f, -23), 1.5f, 1.f};
        for (float x : m) steps.push_back(ldexpf(x, k));
    }
    for (int i = 1; i <= 64; ++i) {
        steps.push_back(float(i));
        steps.push_back(i + 0.5f);
    }
    std::uniform_real_distribution<double> E(-20.0, 20.0);
    for (int i = 0; i < 200; ++i) steps.push_back(float(exp2(E(g))));
    std::uniform_real_distribution<double> Q(-3.0, 26.0);
    std::uniform_int_distribution<int> K(-40000, 40000), U(-3, 3);
    for (float b : steps) {
        if (!fast_step(b)) continue;
        const float r = 1.0f / b;
        for (int i = 0; i < 40000; ++i) {
            float a;
            if (i & 1) {
                a = float((K(g) + 0.5) * double(b));
                for (int u = U(g); u != 0; u += (u > 0 ? -1 : 1)) a = nextafterf(a, u > 0 ? INFINITY : -INFINITY);
            } else {
                a = float(exp2(Q(g)) * double(b) * ((g() & 1) ? 1.0 : -1.0));
            }
            ++checked;
            if (quant_index(a, b, r) != to_index(a / b)) {
                if (bad_q < 5) printf("quant_index(%a, %a) = %d, division gives %d\n", a, b, quant_index(a, b, r), to_index(a / b));
                ++bad_q;
            }
        }
    }
    const bool range = fast_step(0x1p-20f) && fast_step(0x1p20f) && !fast_step(nextafterf(0x1p-20f, 0.f)) &&
                       !fast_step(nextafterf(0x1p20f, INFINITY)) && !fast_step(NAN) && !fast_step(-1.f);
    printf("to_index mismatches %lld, quant_index mismatches %lld of %lld, range %s\n", bad_round, bad_q, checked,
           range ? "ok" : "wrong");
    if (bad_round || bad_q || !range) return 1;
    printf("quant index clean\n");
    return 0;
}

// Quantiser and dequantiser kernels for gfx950 (built without FMA
// contraction; the arithmetic is in ct_quant_stages.h).
//
// Paper section 3.4 (lowpass normalised to [0, 255] and restored at the
// decoder), section 3.5 (division by QPH / QPL, then rounding to an
// integer), section 3.6 (rounding to the nearest integer).
//
// The lowpass min/max is a two-pass reduction without atomics: pass 1 writes
// one (min, max) partial per block of the lowpass; every quantiser tile that
// touches the lowpass reduces its plane's partials with wavefront shuffles,
// so the result does not depend on scheduling.
#include "ct_quant_stages.h"

namespace ct {
namespace {

constexpr int NT = 256;

__global__ __launch_bounds__(NT) void lowpass_partial_kernel(QuantArgs A) {
    __shared__ float red[2 * NT / 64];
    qstage::lowpass_partial<NT>(A, blockIdx.x, red);
}

__global__ __launch_bounds__(NT) void quantize_kernel(QuantArgs A) {
    __shared__ float red[2 * NT / 64];
    qstage::quantize<NT>(A, blockIdx.x, red);
}

__global__ __launch_bounds__(NT) void dequantize_kernel(QuantArgs A) {
    qstage::dequantize<NT>(A, blockIdx.x);
}

unsigned chunks(int64_t n, int batch) {
    return unsigned((n + qstage::CHUNK - 1) / qstage::CHUNK) * unsigned(batch);
}

}  // namespace

hipError_t launch_lowpass_partial(const QuantArgs& a, int batch, hipStream_t st) {
    lowpass_partial_kernel<<<dim3(a.nparts * batch), NT, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_quantize(const QuantArgs& a, int batch, hipStream_t st) {
    quantize_kernel<<<dim3(chunks(a.nq, batch)), NT, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_dequantize(const QuantArgs& a, int batch, hipStream_t st) {
    dequantize_kernel<<<dim3(chunks(a.ncoef, batch)), NT, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace ct

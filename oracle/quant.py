"""Uniform quantiser and dequantiser of the contourlet coefficients.

Paper:
  * section 3.4: the lowpass is normalised to [0, 255] and restored to its
    range at the decoder;
  * section 3.5: every element is divided by a quantisation parameter (QPH
    for the directional subbands, QPL for the lowpass) and rounded to an
    integer; a parameter of 1 leaves the elements unchanged apart from the
    rounding, and a large enough parameter sends every directional element
    to zero;
  * section 3.6: the coefficients are rounded to the nearest integer.

Readings:
  * lowpass normalisation is per plane min-max: mn = min c, mx = max c,
    s = 255 / (mx - mn); if mx == mn then s = 0 and every index is 0;
  * one step per subband (index 0 = lowpass, then the packed subband order);
  * "nearest integer" rounds halves away from zero;
  * indices are int16; values beyond the int16 range saturate and a NaN
    maps to 0 (the paper's 8-bit range needs no clamping in practice);
  * dequantise: directional c = q * step, lowpass c = mn + (q * step) * ((mx - mn) / 255).

Two versions:
  * quantize64 / dequantize64: the FP64 pipeline of the oracle;
  * quantize32 / dequantize32: the same formulas evaluated in IEEE FP32 in a
    fixed operation order, which defines the bit-exact contract for the
    device quantiser given the same FP32 coefficients:
        d = mx - mn; s = 255 / d; t = c - mn; u = t * s; v = u / step
        directional: v = c / step
        q = round_half_away(v)
    round_half_away works on the exact float64 value of the float32 v:
    floor(|v| + 0.5) * sign(v) is exact in float64, whereas float32 |v| + 0.5
    would misround 0.49999997.
"""
import numpy as np

INT16_MIN, INT16_MAX = -32768, 32767


def round_half_away(v):
    """Nearest integer, halves away from zero, in float64; NaN -> 0."""
    v = np.asarray(v, dtype=np.float64)
    r = np.floor(np.abs(v) + 0.5) * np.sign(v)
    return np.where(np.isnan(v), 0.0, r)


def to_int16(r):
    """Saturate a float64 array of integers to int16."""
    return np.clip(r, INT16_MIN, INT16_MAX).astype(np.int16)


def _step_vector(table, steps):
    """Per-coefficient step: steps[s] over the elements of subband s."""
    steps = np.asarray(steps)
    assert steps.shape == (len(table),)
    out = np.empty(table[-1].offset + table[-1].size, dtype=steps.dtype)
    for s, sb in enumerate(table):
        out[sb.offset:sb.offset + sb.size] = steps[s]
    return out


def quantize64(coeffs, steps, table):
    """FP64 quantiser of one plane: returns (int16 indices, (mn, mx))."""
    c = np.asarray(coeffs, dtype=np.float64)
    nlow = table[0].size
    low = c[:nlow]
    mn, mx = float(low.min()), float(low.max())
    s = 0.0 if mx == mn else 255.0 / (mx - mn)
    stepv = _step_vector(table, np.asarray(steps, dtype=np.float64))
    v = np.empty_like(c)
    v[:nlow] = ((low - mn) * s) / stepv[:nlow]
    v[nlow:] = c[nlow:] / stepv[nlow:]
    return to_int16(round_half_away(v)), (mn, mx)


def dequantize64(idx, steps, side, table):
    """FP64 dequantiser of one plane."""
    q = np.asarray(idx, dtype=np.float64)
    mn, mx = side
    stepv = _step_vector(table, np.asarray(steps, dtype=np.float64))
    out = q * stepv
    nlow = table[0].size
    out[:nlow] = mn + (q[:nlow] * stepv[:nlow]) * ((mx - mn) / 255.0)
    return out


def quantize32(coeffs32, steps32, table):
    """FP32 quantiser in the fixed operation order; (int16 indices, (mn, mx))."""
    f = np.float32
    c = np.asarray(coeffs32, dtype=np.float32)
    nlow = table[0].size
    low = c[:nlow]
    mn, mx = f(low.min()), f(low.max())
    d = f(mx - mn)
    s = f(0.0) if mx == mn else f(f(255.0) / d)
    stepv = _step_vector(table, np.asarray(steps32, dtype=np.float32))
    v = np.empty_like(c)
    t = (low - mn).astype(np.float32)
    u = (t * s).astype(np.float32)
    v[:nlow] = (u / stepv[:nlow]).astype(np.float32)
    v[nlow:] = (c[nlow:] / stepv[nlow:]).astype(np.float32)
    return to_int16(round_half_away(v)), (mn, mx)


def dequantize32(idx, steps32, side32, table):
    """FP32 dequantiser: c = q*step; lowpass c = mn + (q*step) * ((mx - mn)/255)."""
    f = np.float32
    q = np.asarray(idx).astype(np.float32)
    mn, mx = f(side32[0]), f(side32[1])
    stepv = _step_vector(table, np.asarray(steps32, dtype=np.float32))
    out = (q * stepv).astype(np.float32)
    nlow = table[0].size
    r = f(f(mx - mn) / f(255.0))
    w = (q[:nlow] * stepv[:nlow]).astype(np.float32)
    out[:nlow] = (mn + (w * r).astype(np.float32)).astype(np.float32)
    return out

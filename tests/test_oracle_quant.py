"""Pins of the quantiser (sections 3.4-3.6)."""
import json
import os

import numpy as np
import pytest

from oracle import ct, quant
from oracle import geometry as geo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
GEOM = (16, 16, 1, [4])


def _table():
    return geo.subband_table(*GEOM)


def test_worked_example():
    with open(os.path.join(GOLDEN, "quant_worked.json")) as f:
        ref = json.load(f)
    table = _table()
    n = table[-1].offset + table[-1].size
    c = np.zeros(n)
    c[:table[0].size] = ref["lowpass_values"]["others"]
    c[ref["lowpass_values"]["index"]] = ref["lowpass_values"]["value"]
    dvals = ref["directional_values"]
    c[table[1].offset:table[1].offset + len(dvals)] = dvals
    for step_d, key in ((1.0, "directional_step1_expected"), (2.0, "directional_step2_expected")):
        for step_l, lkey in ((1.0, "lowpass_expected_q"), (2.0, "lowpass_expected_q_step2")):
            steps = np.array([step_l] + [step_d] * (len(table) - 1))
            for qfun, cast in ((quant.quantize64, np.float64), (quant.quantize32, np.float32)):
                q, (mn, mx) = qfun(c.astype(cast), steps.astype(cast), table)
                assert (mn, mx) == (10.0, 30.0)
                assert list(q[ref["lowpass_values"]["index"]]) == ref[lkey]
                assert list(q[table[1].offset:table[1].offset + len(dvals)]) == ref[key]


def test_ties_round_away_from_zero():
    v = np.array([0.5, 1.5, 2.5, -0.5, -1.5, -2.5, 0.49999997, -0.49999997, 1e9, -1e9, np.nan])
    r = quant.round_half_away(v.astype(np.float32))
    assert list(quant.to_int16(r)) == [1, 2, 3, -1, -2, -3, 0, 0, 32767, -32768, 0]


def test_step_one_is_plain_rounding():
    """Section 3.5: a parameter of 1 alters nothing beyond the integer rounding."""
    table = geo.subband_table(64, 64, 2, [8, 4])
    c = ct.forward(np.random.default_rng(31).uniform(0, 255, (64, 64)), 2, [8, 4])
    q, _ = quant.quantize64(c, np.ones(len(table)), table)
    n_low = table[0].size
    np.testing.assert_array_equal(q[n_low:], quant.round_half_away(c[n_low:]))
    assert np.abs(q[n_low:] - c[n_low:]).max() <= 0.5


def test_large_step_zeroes_directional():
    """Section 3.5: a large enough QPH sends every directional element to 0."""
    table = geo.subband_table(64, 64, 2, [8, 4])
    c = ct.forward(np.random.default_rng(32).uniform(0, 255, (64, 64)), 2, [8, 4])
    n_low = table[0].size
    big = 2.0 * np.abs(c[n_low:]).max() + 1.0
    q, _ = quant.quantize64(c, np.array([1.0] + [big] * (len(table) - 1)), table)
    assert np.all(q[n_low:] == 0)


def test_lowpass_normalised_to_0_255():
    """Section 3.4: the lowpass is mapped to [0, 255]; with step 1 the indices span it."""
    table = geo.subband_table(64, 64, 2, [8, 4])
    c = ct.forward(np.random.default_rng(33).uniform(0, 255, (64, 64)), 2, [8, 4])
    q, (mn, mx) = quant.quantize64(c, np.ones(len(table)), table)
    low = q[:table[0].size]
    assert low.min() == 0 and low.max() == 255
    # restored to the original range within half a quantisation bin
    back = quant.dequantize64(q, np.ones(len(table)), (mn, mx), table)
    assert np.abs(back[:table[0].size] - c[:table[0].size]).max() <= 0.5 * (mx - mn) / 255 + 1e-9


def test_constant_lowpass_gives_zero_indices():
    table = _table()
    n = table[-1].offset + table[-1].size
    c = np.zeros(n, dtype=np.float32)
    c[:table[0].size] = 42.0
    q, (mn, mx) = quant.quantize32(c, np.full(len(table), 3.0, np.float32), table)
    assert mn == mx == 42.0 and np.all(q == 0)
    back = quant.dequantize32(q, np.full(len(table), 3.0, np.float32), (mn, mx), table)
    assert np.all(back[:table[0].size] == 42.0)


@pytest.mark.parametrize("step", [1.0, 4.0, 16.0, 37.0])
def test_requantising_dequantised_indices_is_identity(step):
    table = geo.subband_table(64, 64, 2, [8, 4])
    c = ct.forward(np.random.default_rng(34).uniform(0, 255, (64, 64)), 2, [8, 4]).astype(np.float32)
    steps = np.full(len(table), step, np.float32)
    q, side = quant.quantize32(c, steps, table)
    back = quant.dequantize32(q, steps, side, table)
    q2, side2 = quant.quantize32(back, steps, table)
    # the lowpass min and max are themselves reconstructed exactly when they
    # are bin centres; compare on the directional part, and on the lowpass
    # up to one bin where the reconstructed range may differ by rounding
    n_low = table[0].size
    np.testing.assert_array_equal(q2[n_low:], q[n_low:])
    assert np.abs(q2[:n_low].astype(int) - q[:n_low]).max() <= 1


def test_fp32_twin_matches_fp64_away_from_ties():
    table = geo.subband_table(64, 64, 2, [8, 4])
    c = ct.forward(np.random.default_rng(35).uniform(0, 255, (64, 64)), 2, [8, 4])
    steps = np.random.default_rng(36).integers(4, 65, len(table)).astype(np.float64)
    q64, _ = quant.quantize64(c, steps, table)
    q32, _ = quant.quantize32(c.astype(np.float32), steps.astype(np.float32), table)
    mismatch = np.mean(q64 != q32)
    assert mismatch < 1e-3
    assert np.abs(q64.astype(int) - q32).max() <= 1

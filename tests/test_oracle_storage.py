"""Pins of the FP8 (E4M3) storage rounding of the oracle (CPU).

The oracle builds the rounding from the format's definition (a table of the
codes and their values, nearest value, ties to the even code).  It is pinned
here to the OCP E4M3 code points, to torch's own float8_e4m3fn conversion
(an independent implementation) and to the scale rule's invariants."""
import math

import numpy as np
import pytest
import torch

from oracle.storage import (E4M3_MAX, e4m3_round, e4m3_value, item_exponent,
                            round_fp8_items)


def test_e4m3_code_points():
    """Values fixed by the format: bias 7, 3 fraction bits, S.1111.111 NaN."""
    assert e4m3_value(0x00) == 0.0
    assert e4m3_value(0x01) == 2.0 ** -9           # smallest subnormal
    assert e4m3_value(0x07) == 7 * 2.0 ** -9       # largest subnormal
    assert e4m3_value(0x08) == 2.0 ** -6           # smallest normal
    assert e4m3_value(0x38) == 1.0
    assert e4m3_value(0x3C) == 1.5
    assert e4m3_value(0x7E) == 448.0 == E4M3_MAX   # largest finite
    assert math.isnan(e4m3_value(0x7F)) and math.isnan(e4m3_value(0xFF))
    assert math.copysign(1.0, e4m3_value(0x80)) == -1.0 and e4m3_value(0x80) == 0.0
    assert e4m3_value(0xB8) == -1.0


def test_e4m3_round_matches_torch():
    """Random values over the whole finite range, small values near the
    subnormals, and every midpoint between neighbouring codes (ties), both
    signs: equal to torch's float8_e4m3fn conversion."""
    rng = np.random.default_rng(0)
    vals = np.array([e4m3_value(c) for c in range(0x7F)])
    mids = 0.5 * (vals[1:] + vals[:-1])
    x = np.concatenate([rng.uniform(-448, 448, 50000), rng.normal(0, 1e-2, 20000),
                        rng.normal(0, 1e-3, 5000), mids, -mids, vals, -vals])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = e4m3_round(x32.astype(np.float64))
    assert np.array_equal(got, ref)
    # ties go to the even code
    assert e4m3_round(np.array([1.0625]))[0] == 1.0      # between 1.0 (0x38) and 1.125 (0x39)
    assert e4m3_round(np.array([1.1875]))[0] == 1.25     # between 1.125 (0x39) and 1.25 (0x3A)


def test_e4m3_saturation_and_non_finite():
    r = e4m3_round(np.array([448.0, 463.9, 464.0, 1e6, -500.0, np.inf, -np.inf, np.nan]))
    assert np.array_equal(r[:5], [448.0, 448.0, 448.0, 448.0, -448.0])
    assert np.all(np.isnan(r[5:]))


def test_e4m3_relative_error_bound():
    """Normal range: |round(v) - v| <= 2^-4 |v| (half a step of 3 fraction bits)."""
    v = np.random.default_rng(1).uniform(2.0 ** -6, 448, 100000) * np.random.default_rng(2).choice([-1, 1], 100000)
    assert np.all(np.abs(e4m3_round(v) - v) <= 2.0 ** -4 * np.abs(v))


@pytest.mark.parametrize("amp", [1e-30, 3e-5, 1.0, 7.0, 255.9, 1e4, 3e30])
def test_item_scale_rule(amp):
    """The scale puts the item's largest magnitude in [128, 256): values far
    below saturation, and the same relative error at any amplitude."""
    rng = np.random.default_rng(3)
    y = (rng.normal(0, 1, (2, 3, 5, 40)) * amp).astype(np.float32)
    for b in range(2):
        e = item_exponent(y[b])
        a = np.max(np.abs(y[b].astype(np.float64))) * 2.0 ** e
        assert 128.0 <= a < 256.0
    yr = round_fp8_items(y)
    big = np.abs(y) >= np.max(np.abs(y)) * 2.0 ** -12   # well inside the normal range after scaling
    rel = np.abs(yr - y)[big] / np.abs(y.astype(np.float64))[big]
    assert np.max(rel) <= 2.0 ** -4
    # scale-invariant: the same data at another amplitude rounds to the same pattern
    y2 = (y.astype(np.float64) * 2.0 ** 20).astype(np.float32)
    if np.all(np.isfinite(y2)) and np.max(np.abs(y2)) < 1e38:
        assert np.array_equal(round_fp8_items(y2) * 2.0 ** -20, yr)


def test_item_scale_special_items():
    y = np.zeros((3, 2, 2, 8), np.float32)
    y[1, 0, 0, 3] = np.nan
    y[1, 1, 1, 1] = 2.0
    y[2] = -1e-3
    assert item_exponent(y[0]) == 0 and item_exponent(y[1]) == 0
    r = round_fp8_items(y)
    assert np.all(r[0] == 0.0)
    assert np.isnan(r[1, 0, 0, 3]) and r[1, 1, 1, 1] == 2.0
    # -1e-3 scaled into [128, 256): 1e-3 = 0.512 * 2^-9, e = 17, 131.07 -> 128
    assert item_exponent(y[2]) == 17 and np.all(r[2] == -128.0 * 2.0 ** -17)

"""What a reduced-precision workspace holds: the FP8 (e4m3) storage form.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper stores channel data in FP16 to halve the bytes moved (Sec. 3.3) and
names lower-precision storage as a future direction (Sec. 5).  The FP8 form
stores every sample in the OCP "E4M3" 8-bit format (1 sign bit, 4 exponent
bits with bias 7, 3 fraction bits; no infinities, the all-ones pattern of
each sign is NaN, largest finite magnitude 448).  Values are rounded to the
nearest representable value, ties to the even code (the code whose last
fraction bit is 0), and finite magnitudes beyond 448 saturate to 448.

Each batch item is first scaled by a power of two 2^e chosen from its largest
magnitude A: A = f 2^x with f in [0.5, 1) gives e = 8 - x, so that A 2^e lies
in [128, 256) (A = 0 or a non-finite A gives e = 0).  The stored value of a
sample s is then round(s 2^e) 2^-e, and the beamformed output of the item is
the sum over these values.

This module writes that rounding out from the format's definition: it lists
the 127 non-negative finite codes with their values and picks the nearest one.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def e4m3_value(code: int) -> float:
    """Value of an E4M3 code (0..255); NaN for the two NaN codes."""
    sign = -1.0 if code & 0x80 else 1.0
    e = (code >> 3) & 0xF
    m = code & 0x7
    if e == 0xF and m == 0x7:
        return float("nan")
    if e == 0:
        return sign * m * 2.0 ** -9            # subnormal: m/8 * 2^(1-7)
    return sign * (1.0 + m / 8.0) * 2.0 ** (e - 7)


def _table():
    codes = np.arange(0, 0x7F)                 # 0x00 .. 0x7E: the finite non-negative codes
    vals = np.array([e4m3_value(int(c)) for c in codes])
    assert np.all(np.diff(vals) > 0)
    return codes, vals


_CODES, _VALS = _table()


def e4m3_round(a: np.ndarray) -> np.ndarray:
    """Round (float64) values to E4M3: nearest value, ties to the even code,
    saturation at +-448, NaN for NaN and +-inf.  Returns float64 values."""
    a = np.asarray(a, np.float64)
    mag = np.abs(a)
    i = np.searchsorted(_VALS, np.minimum(mag, E4M3_MAX), side="left")  # first value >= mag
    i = np.clip(i, 0, len(_VALS) - 1)
    lo = np.clip(i - 1, 0, len(_VALS) - 1)
    up, dn = _VALS[i], _VALS[lo]
    d_up, d_dn = up - np.minimum(mag, E4M3_MAX), np.minimum(mag, E4M3_MAX) - dn
    take_up = (d_up < d_dn) | ((d_up == d_dn) & (_CODES[i] % 2 == 0))
    take_up |= i == 0
    r = np.where(take_up, up, dn)
    r = np.where(np.isfinite(a), np.copysign(r, a), np.nan)
    return r


def item_exponent(y_item: np.ndarray) -> int:
    """Scale exponent e of one batch item (A 2^e in [128, 256))."""
    amax = float(np.max(np.abs(np.asarray(y_item, np.float64)))) if np.size(y_item) else 0.0
    if not np.isfinite(amax) or amax == 0.0:
        return 0
    _, x = np.frexp(amax)
    return int(8 - x)


def round_fp8_items(y: np.ndarray) -> np.ndarray:
    """The values an FP8 workspace holds for y[B, ...] (float32 input; one
    scale per leading index).  Returns float64."""
    y = np.asarray(y, np.float32)
    out = np.empty(y.shape, np.float64)
    for b in range(y.shape[0]):
        e = item_exponent(y[b])
        out[b] = np.ldexp(e4m3_round(np.ldexp(y[b].astype(np.float64), e)), -e)
    return out

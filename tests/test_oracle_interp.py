"""Pins of the oracle's higher-order interpolation (the paper allows other
schemes than linear after Eq. (2); reading R15: the four-point Lagrange cubic
through samples k-1 .. k+2).

The four tap weights at a fractional position are fixed uniquely by
reproducing the polynomials 1, k, k^2 and k^3, so exact reproduction of random
cubics pins all of them; the adjoint is pinned by the dot-product test, zero
padding by comparison with explicit zeros, and the benefit of the higher order
by the error on a sampled sinusoid.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.test_oracle_pins import _f_and_w, _small_geometry


def _cubic_data(g, coef):
    k = np.arange(g.K, dtype=np.float64)
    p = coef[0] + coef[1] * k + coef[2] * k ** 2 + coef[3] * k ** 3
    return np.broadcast_to(p, (1, g.Q, g.M, g.K)).copy(), p


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cubic_reproduces_cubic_polynomials(seed):
    g = _small_geometry()
    f, w = _f_and_w(g)
    assert f.min() > 2 and f.max() < g.K - 3                   # all four taps in range
    rng = np.random.default_rng(seed)
    coef = rng.normal(size=4) * np.array([1.0, 0.1, 1e-3, 1e-6])
    y, _ = _cubic_data(g, coef)
    x = oracle.forward(y, g, interp="cubic")[0]
    expect = np.sum(w * (coef[0] + coef[1] * f + coef[2] * f ** 2 + coef[3] * f ** 3), axis=(0, 1))
    np.testing.assert_allclose(x, expect, rtol=1e-11, atol=1e-11 * np.abs(expect).max())
    # linear interpolation does not reproduce the cubic part
    if abs(coef[2]) > 1e-5:
        xl = oracle.forward(y, g)[0]
        assert np.max(np.abs(xl - expect)) > 1e3 * np.max(np.abs(x - expect))


def test_cubic_interpolates_the_samples():
    """At integer f the interpolant is the sample itself (weights 0, 1, 0, 0)."""
    c, fs, K = 1500.0, 30e6, 64
    y = np.random.default_rng(3).normal(size=(1, 1, 1, K))
    base = 0.003 * fs / c                                     # D_rx = 3 mm
    for j in (1, 17, 40, K - 3):
        g = synth.Geometry(elem_pos=np.zeros((1, 3)), elem_normal=None,
                           tx_kind=np.array([synth.TX_NONE], np.int32), tx_vec=np.zeros((1, 3)),
                           tx_offset=np.zeros(1), grid_origin=(0.0, 0.0, 0.003),
                           grid_spacing=(1e-4,) * 3, grid_dims=(1, 1, 1), num_samples=K, c=c, fs=fs,
                           t0=(base - j) / fs)
        assert oracle.forward(y, g, interp="cubic")[0, 0] == pytest.approx(y[0, 0, 0, j], abs=1e-9)


def test_cubic_zero_padding_equals_explicit_zeros():
    """Taps outside [0, K) read zero: the same image from a record extended by
    8 explicit zeros on each side (time origin moved by 8 samples)."""
    g0 = _small_geometry(K=400)
    f0, _ = _f_and_w(g0)
    rng = np.random.default_rng(4)
    y = rng.normal(size=(1, g0.Q, g0.M, g0.K))
    yp = np.concatenate([np.zeros((1, g0.Q, g0.M, 8)), y, np.zeros((1, g0.Q, g0.M, 8))], axis=-1)
    # time origins that put the taps across the first and across the last samples
    for shift in (f0.min() + 1.5, f0.max() - g0.K - 1.0):
        g = g0.replace(t0=shift / g0.fs)
        f, _ = _f_and_w(g)
        assert f.min() < 1 or f.max() > g.K - 3
        gp = g.replace(num_samples=g.K + 16, t0=g.t0 - 8 / g.fs)
        np.testing.assert_allclose(oracle.forward(y, g, interp="cubic"),
                                   oracle.forward(yp, gp, interp="cubic"), rtol=1e-9, atol=1e-10)


def test_cubic_adjoint_dot_product():
    g = _small_geometry()
    f0, _ = _f_and_w(g)
    g = g.replace(t0=(f0.min() + 1.5) / g.fs)                # some taps off the record
    rng = np.random.default_rng(5)
    y = rng.normal(size=(2, g.Q, g.M, g.K))
    x = rng.normal(size=(2, g.N))
    wtx = rng.uniform(0.2, 1.0, size=(g.Q, g.N))
    lhs = np.sum(oracle.forward(y, g, w_tx=wtx, interp="cubic") * x)
    rhs = np.sum(y * oracle.adjoint(x, g, w_tx=wtx, interp="cubic"))
    assert abs(lhs) > 1.0
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_cubic_beats_linear_on_a_sampled_carrier():
    """A 7.5 MHz sinusoid sampled at 30 MHz (four samples per period), read at
    the fractional indices of a geometry: the cubic interpolant's error is far
    below the linear one's."""
    g = _small_geometry(K=600)
    f, w = _f_and_w(g)
    fc = 7.5e6
    k = np.arange(g.K)
    y = np.broadcast_to(np.sin(2 * np.pi * fc * k / g.fs), (1, g.Q, g.M, g.K)).copy()
    exact = np.sum(w * np.sin(2 * np.pi * fc * f / g.fs), axis=(0, 1))
    e_lin = np.linalg.norm(oracle.forward(y, g)[0] - exact) / np.linalg.norm(exact)
    e_cub = np.linalg.norm(oracle.forward(y, g, interp="cubic")[0] - exact) / np.linalg.norm(exact)
    assert e_cub < 0.5 * e_lin

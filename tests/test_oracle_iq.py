"""Pins of the complex baseband (IQ) beamformer of the oracle (CPU)."""
import numpy as np
import pytest

import oracle
import synth
from oracle.iq import demodulate, forward_iq
from tests import greens


def _one_voxel_geometry(elem, vox, K=2048, fs=30e6, t0=0.0, c=1540.0):
    return synth.Geometry(elem_pos=np.asarray(elem, float)[None], elem_normal=None,
                          tx_kind=np.array([synth.TX_PLANE], np.int32),
                          tx_vec=np.array([[0.0, 0.0, 1.0]]), tx_offset=np.zeros(1),
                          grid_origin=tuple(vox), grid_spacing=(1e-4,) * 3, grid_dims=(1, 1, 1),
                          num_samples=K, c=c, fs=fs, t0=t0)


def test_zero_carrier_is_two_real_beamformers():
    g = synth.cfg2(dims=(6, 5, 4), n_side=4).replace(num_samples=900)
    rng = np.random.default_rng(0)
    yi = rng.normal(size=(2, g.Q, g.M, g.K))
    yq = rng.normal(size=(2, g.Q, g.M, g.K))
    x = forward_iq(yi + 1j * yq, g, fc=0.0)
    ref = oracle.forward(yi, g) + 1j * oracle.forward(yq, g)
    assert np.allclose(x, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("fc", [7.5e6, 5.0e6])
def test_hand_phase_on_a_3_4_5_triangle(fc):
    """Element at the origin, plane wave at 0 deg, voxel at (3, 0, 4) mm:
    transmit path 4 mm + receive path 5 mm = 9 mm.  Constant baseband data
    (interpolation exact) gives x = exp(i 2 pi fc 9 mm / c)."""
    c = 1540.0
    g = _one_voxel_geometry((0.0, 0.0, 0.0), (3e-3, 0.0, 4e-3), c=c)
    y = np.ones((1, 1, 1, g.K), np.complex128)
    x = forward_iq(y, g, fc=fc)
    assert x[0, 0] == pytest.approx(np.exp(2j * np.pi * fc * 9e-3 / c), abs=1e-12)


def test_baseband_beamformer_matches_the_analytic_rf_one():
    """A point scatterer (frequency-domain Green's-function simulation, 480 MHz
    sampling): beamforming the demodulated IQ records with phase rotation gives
    the analytic-RF beamformer's value at the scatterer (within the linear
    interpolation error of the RF carrier, 0.1 % at 64 samples per period) and
    the same envelope peak along a line of voxels through it."""
    fs, c, fc = 480e6, 1540.0, 7.5e6
    sigma = synth.pulse_sigma()
    elems = synth.matrix_array(4, 0.3e-3)
    scat = np.array([0.2e-3, -0.1e-3, 6.0e-3])
    t0, K = 5.0e-6, 4096
    u = np.array([0.0, 0.0, 1.0])
    ya = greens.simulate(elems, scat[None], np.array([1.0]), ("plane", u), c, fs, t0, K, fc, sigma,
                         nfft=32768, analytic_out=True)                       # [M, K] complex
    g = synth.Geometry(elem_pos=elems, elem_normal=None, tx_kind=np.array([synth.TX_PLANE], np.int32),
                       tx_vec=u[None], tx_offset=np.zeros(1),
                       grid_origin=(scat[0], scat[1], scat[2] - 10 * 0.02e-3),
                       grid_spacing=(1e-4, 1e-4, 0.02e-3), grid_dims=(1, 1, 21),
                       num_samples=K, c=c, fs=fs, t0=t0)
    x_rf = forward_iq(ya[None, None], g, fc=0.0)[0]
    x_iq = forward_iq(demodulate(ya, fs, t0, fc)[None, None], g, fc=fc)[0]
    i0 = 10
    assert abs(x_iq[i0] - x_rf[i0]) <= 1e-2 * abs(x_rf[i0])
    assert np.argmax(np.abs(x_iq)) == np.argmax(np.abs(x_rf)) == i0


def test_adjoint_iq_dot_product():
    """adjoint_iq is the transpose of forward_iq under Re(sum a conj(b))."""
    from oracle.iq import adjoint_iq
    g = synth.cfg2(dims=(6, 5, 4), n_side=4).replace(num_samples=900)
    rng = np.random.default_rng(7)
    y = rng.normal(size=(2, g.Q, g.M, g.K)) + 1j * rng.normal(size=(2, g.Q, g.M, g.K))
    gx = rng.normal(size=(2, g.N)) + 1j * rng.normal(size=(2, g.N))
    lhs = np.sum(forward_iq(y, g, fc=7.5e6) * np.conj(gx)).real
    rhs = np.sum(y * np.conj(adjoint_iq(gx, g, fc=7.5e6))).real
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_iq_zero_carrier_is_two_real_adjoints():
    from oracle.iq import adjoint_iq
    g = synth.cfg2(dims=(6, 5, 4), n_side=4).replace(num_samples=900)
    rng = np.random.default_rng(8)
    gi, gq = rng.normal(size=(2, g.N)), rng.normal(size=(2, g.N))
    gy = adjoint_iq(gi + 1j * gq, g, fc=0.0)
    ref = oracle.adjoint(gi, g) + 1j * oracle.adjoint(gq, g)
    assert np.allclose(gy, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("fc", [7.5e6, 5.0e6])
def test_adjoint_iq_hand_phase_on_a_3_4_5_triangle(fc):
    """The 3-4-5 voxel of the forward pin: a unit upstream gradient lands on
    the two taps of the 9 mm path with weights summing to
    exp(-i 2 pi fc 9 mm / c)."""
    from oracle.iq import adjoint_iq
    c = 1540.0
    g = _one_voxel_geometry((0.0, 0.0, 0.0), (3e-3, 0.0, 4e-3), c=c)
    gy = adjoint_iq(np.ones((1, 1), np.complex128), g, fc=fc)
    assert np.count_nonzero(gy) <= 2
    assert gy.sum() == pytest.approx(np.exp(-2j * np.pi * fc * 9e-3 / c), abs=1e-12)


def test_dforward_dc_iq_vs_finite_differences():
    """Central differences of forward_iq in c with a step too small for any
    tap index to change (checked): the interpolant is linear in f between
    integers and the phase is smooth in c, so the quotient equals the
    analytic derivative up to rounding."""
    from oracle.iq import dforward_dc_iq
    g = synth.sub_grid(synth.cfg5(), (28, 28, 20), (4, 4, 4))
    rng = np.random.default_rng(9)
    y = rng.normal(size=(1, g.Q, g.M, g.K)) + 1j * rng.normal(size=(1, g.Q, g.M, g.K))
    fc, h = 7.5e6, 2e-6
    p = oracle.voxel_positions(g)
    path = oracle.transmit_path(g, p)[:, None, :] + oracle.receive_path(g, p)[None, :, :]
    k_lo = np.floor(oracle.fractional_index(path, 0.0, g.c - h, g.fs, g.t0))
    k_hi = np.floor(oracle.fractional_index(path, 0.0, g.c + h, g.fs, g.t0))
    assert np.array_equal(k_lo, k_hi)
    d = dforward_dc_iq(y, g, fc)
    fd = (forward_iq(y, g, fc, c=g.c + h) - forward_iq(y, g, fc, c=g.c - h)) / (2 * h)
    assert np.linalg.norm(fd - d) / np.linalg.norm(d) < 1e-7
    # the phase term matters: without it the quotient is far off
    d_real = oracle.dforward_dc(y.real, g) + 1j * oracle.dforward_dc(y.imag, g)
    assert np.linalg.norm(fd - d_real) / np.linalg.norm(d) > 0.1


def test_dforward_dc_iq_zero_carrier_is_two_real_derivatives():
    from oracle.iq import dforward_dc_iq
    g = synth.cfg2(dims=(6, 5, 4), n_side=4).replace(num_samples=900)
    rng = np.random.default_rng(10)
    yi, yq = rng.normal(size=(2, g.Q, g.M, g.K)), rng.normal(size=(2, g.Q, g.M, g.K))
    d = dforward_dc_iq(yi + 1j * yq, g, fc=0.0)
    ref = oracle.dforward_dc(yi, g) + 1j * oracle.dforward_dc(yq, g)
    assert np.allclose(d, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("fc", [7.5e6, 5.0e6])
def test_dforward_dc_iq_hand_value_on_a_3_4_5_triangle(fc):
    """Constant baseband data on the 3-4-5 voxel: x(c) = exp(i 2 pi fc L / c)
    with L = 9 mm, so dx/dc = -i 2 pi fc L / c^2 x (the slope term vanishes),
    and the loss gradient for gx = 1 - 2i is Re(conj(gx) dx/dc)."""
    from oracle.iq import dforward_dc_iq, grad_sound_speed_iq
    c, L = 1540.0, 9e-3
    g = _one_voxel_geometry((0.0, 0.0, 0.0), (3e-3, 0.0, 4e-3), c=c)
    y = np.ones((1, 1, 1, g.K), np.complex128)
    x = np.exp(2j * np.pi * fc * L / c)
    want = -2j * np.pi * fc * L / c ** 2 * x
    assert dforward_dc_iq(y, g, fc)[0, 0] == pytest.approx(want, rel=1e-12)
    gx = np.array([[1.0 - 2.0j]])
    assert grad_sound_speed_iq(y, gx, g, fc) == pytest.approx((np.conj(gx[0, 0]) * want).real, rel=1e-12)

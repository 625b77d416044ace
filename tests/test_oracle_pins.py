"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  None of them re-types the oracle's formula:
they use hand-evaluated exact geometries, an independent wave-physics
simulator, closed forms of the interpolant, invariances of the operator and
finite differences.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests import greens

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _single(elem, voxel, kind, vec, offset, c, fs, t0, K=1024, apod=synth.APOD_UNIFORM, F=1.0,
            normal=None):
    """A geometry with one element, one transmit and one voxel."""
    return synth.Geometry(
        elem_pos=np.asarray([elem], float),
        elem_normal=None if normal is None else np.asarray([normal], float),
        tx_kind=np.asarray([kind], np.int32), tx_vec=np.asarray([vec], float),
        tx_offset=np.asarray([offset], float), grid_origin=tuple(voxel),
        grid_spacing=(1e-4, 1e-4, 1e-4), grid_dims=(1, 1, 1), num_samples=K, c=c, fs=fs,
        t0=t0, apod=apod, f_number=F)


# ---------------------------------------------------------------------------
# Eq. (1) and its footnote: exact hand-evaluated delays
# ---------------------------------------------------------------------------

def test_delay_hand_cases():
    spec = json.load(open(os.path.join(GOLDEN, "delay_cases.json")))
    cm = spec["common"]
    for case in spec["cases"]:
        g = _single(cm["element"], cm["voxel"], case["kind"], case["vec"], case["offset"],
                    cm["c"], cm["fs"], case["t0"])
        p = oracle.voxel_positions(g)
        d_tx = oracle.transmit_path(g, p)[0, 0]
        d_rx = oracle.receive_path(g, p)[0, 0]
        f = oracle.fractional_index(d_tx, d_rx, g.c, g.fs, g.t0)
        assert d_tx == pytest.approx(case["d_tx"], abs=1e-15), case["name"]
        assert d_rx == pytest.approx(case["d_rx"], abs=1e-15), case["name"]
        assert f == pytest.approx(case["f"], abs=1e-9), case["name"]


def test_single_term_forward_by_hand():
    """M = Q = N = 1: x = w ((1-a) y[k] + a y[k+1]) with k, a from f = 179.7."""
    g = _single([0, 0, 0], [0.003, 0, 0.004], synth.TX_PLANE, [0, 0, 1], 0.0, 1500.0, 30e6, 1e-8,
                K=256)
    y = np.zeros((1, 1, 1, 256))
    y[0, 0, 0, 179] = 2.0
    y[0, 0, 0, 180] = -1.0
    x = oracle.forward(y, g)
    assert x[0, 0] == pytest.approx(0.3 * 2.0 + 0.7 * -1.0, abs=1e-9)
    # a transmit weight scales the single term
    x2 = oracle.forward(y, g, w_tx=np.array([[0.25]]))
    assert x2[0, 0] == pytest.approx(0.25 * x[0, 0], abs=1e-12)


# ---------------------------------------------------------------------------
# Physics: the echo of a point scatterer arrives at the oracle's f
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("incident", ["point", "plane0", "plane_steered"])
def test_echo_arrival_matches_delay(incident):
    fs, c, fc = 30e6, 1540.0, 7.5e6
    sigma = synth.pulse_sigma()
    elems = synth.matrix_array(4, 0.3e-3)
    scat = np.array([0.4e-3, -0.25e-3, 6.1e-3])
    t0 = 2.0e-6
    if incident == "point":
        v = np.array([1.0e-3, 0.5e-3, -10e-3])
        kind, vec, inc = synth.TX_DIVERGING, v, ("point", v)
    elif incident == "plane0":
        u = np.array([0.0, 0.0, 1.0])
        kind, vec, inc = synth.TX_PLANE, u, ("plane", u)
    else:
        u = synth.plane_wave(12.0, -7.0)
        kind, vec, inc = synth.TX_PLANE, u, ("plane", u)
    K = 512
    y = greens.simulate(elems, scat[None], np.array([1.0]), inc, c, fs, t0, K, fc, sigma,
                        nfft=8192, analytic_out=True)
    g = synth.Geometry(elem_pos=elems, elem_normal=None, tx_kind=np.array([kind], np.int32),
                       tx_vec=np.asarray(vec, float)[None], tx_offset=np.zeros(1),
                       grid_origin=tuple(scat), grid_spacing=(1e-4,) * 3, grid_dims=(1, 1, 1),
                       num_samples=K, c=c, fs=fs, t0=t0)
    p = oracle.voxel_positions(g)
    f = oracle.fractional_index(oracle.transmit_path(g, p), oracle.receive_path(g, p), c, fs, t0)
    for m in range(elems.shape[0]):
        assert greens.peak_time_samples(y[m]) == pytest.approx(f[m, 0], abs=0.02)


def test_focusing_at_scatterer_voxels():
    """cfg1 geometry sampled at 120 MHz (so that linear interpolation of the
    RF carrier loses little); each scatterer alone at a voxel centre, data from
    plane-wave physics; the envelope peaks at that voxel."""
    g = synth.cfg1().replace(fs=120e6, num_samples=1024)
    rng = np.random.default_rng(11)
    idx = np.stack([rng.integers(4, 12, 3), rng.integers(4, 12, 3), rng.integers(3, 10, 3)], 1)
    for (ix, iy, iz) in idx:
        pos = synth.voxel_centre(g, ix, iy, iz)[None]
        ya = greens.simulate(g.elem_pos, pos, np.array([1.0]), ("plane", g.tx_vec[0]), g.c,
                             g.fs, g.t0, g.K, synth.FC, synth.pulse_sigma(), nfft=4096,
                             analytic_out=True)
        y2 = np.stack([ya.real, ya.imag])[:, None]            # two real lanes = Re, Im
        sub = synth.sub_grid(g, (ix - 2, iy - 2, iz - 2), (5, 5, 5))
        x = oracle.forward(y2, sub)
        env = np.hypot(x[0], x[1])
        assert int(np.argmax(env)) == 2 + 5 * (2 + 5 * 2)


# ---------------------------------------------------------------------------
# Interpolation and indexing: closed forms (the sentence after Eq. (2))
# ---------------------------------------------------------------------------

def _small_geometry(kind=synth.TX_DIVERGING, apod=synth.APOD_HANN, K=400):
    g = synth.cfg2(dims=(6, 5, 4), n_side=4)
    g = g.replace(num_samples=K, apod=apod, f_number=0.8,
                  tx_kind=np.array([kind, synth.TX_PLANE], np.int32),
                  tx_vec=np.array([[0.5e-3, -0.3e-3, -9e-3], synth.plane_wave(5.0, -3.0)]),
                  tx_offset=np.array([9e-3, 0.0]))
    return g


def _f_and_w(g):
    p = oracle.voxel_positions(g)
    f = oracle.fractional_index(oracle.transmit_path(g, p)[:, None, :],
                                oracle.receive_path(g, p)[None, :, :], g.c, g.fs, g.t0)
    w = oracle.receive_weight(g, p)[None, :, :] * np.ones((g.Q, 1, 1))
    return f, w                                                     # [Q, M, N]


def test_linear_ramp_is_interpolated_exactly():
    g = _small_geometry()
    f, w = _f_and_w(g)
    assert f.min() > 1 and f.max() < g.K - 2                        # both taps in range
    a, b = 0.37, -5.0
    y = np.broadcast_to(a * np.arange(g.K) + b, (1, g.Q, g.M, g.K))
    x = oracle.forward(y, g)[0]
    expect = np.sum(w * (a * f + b), axis=(0, 1))
    np.testing.assert_allclose(x, expect, rtol=1e-12, atol=1e-10)


def test_delta_selects_the_two_tap_weights():
    g = _small_geometry(apod=synth.APOD_UNIFORM)
    f, w = _f_and_w(g)
    q, m, n = 1, 5, 17
    k = int(np.floor(f[q, m, n]))
    alpha = f[q, m, n] - k
    for j, coef in ((k, 1 - alpha), (k + 1, alpha)):
        y = np.zeros((1, g.Q, g.M, g.K))
        y[0, q, m, j] = 1.0
        x = oracle.forward(y, g)[0]
        assert x[n] == pytest.approx(coef, abs=1e-12)


def test_constant_data_sums_weights():
    g = _small_geometry()
    f, w = _f_and_w(g)
    y = np.ones((1, g.Q, g.M, g.K))
    x = oracle.forward(y, g)[0]
    np.testing.assert_allclose(x, w.sum(axis=(0, 1)), rtol=1e-12)


def test_zero_padding_at_both_ends():
    """f in [K-1, K): w (1-a) y[K-1]; f in [-1, 0): w a y[0]; beyond: 0."""
    c, fs, K = 1500.0, 30e6, 64
    y = np.zeros((1, 1, 1, K))
    y[0, 0, 0, 0] = 3.0
    y[0, 0, 0, K - 1] = 5.0
    y[0, 0, 0, 1:K - 1] = 100.0
    base = 0.003 * fs / c                                   # D_rx = 3 mm -> 60 samples
    for f_target, expect in ((K - 1 + 0.25, 0.75 * 5.0), (-0.25, 0.75 * 3.0),
                             (-1.5, 0.0), (K + 0.5, 0.0), (K - 1.0, 5.0)):
        t0 = (base - f_target) / fs
        g = _single([0, 0, 0], [0, 0, 0.003], synth.TX_NONE, [0, 0, 0], 0.0, c, fs, t0, K=K)
        x = oracle.forward(y, g)
        assert x[0, 0] == pytest.approx(expect, abs=1e-9), f_target


# ---------------------------------------------------------------------------
# Receive weight (reading R5): special values
# ---------------------------------------------------------------------------

def test_hann_weight_special_values():
    F = 1.5
    z = 0.006
    a = z / (2 * F)
    for rho, expect in ((0.0, 1.0), (a / 2, 0.5), (a / 3, 0.75), (a, 0.0), (1.2 * a, 0.0)):
        g = _single([0, 0, 0], [rho, 0, z], synth.TX_NONE, [0, 0, 0], 0, 1540, 30e6, 0,
                    apod=synth.APOD_HANN, F=F)
        w = oracle.receive_weight(g, oracle.voxel_positions(g))[0, 0]
        assert w == pytest.approx(expect, abs=1e-12)
    # behind the element
    g = _single([0, 0, 0], [0, 0, -z], synth.TX_NONE, [0, 0, 0], 0, 1540, 30e6, 0,
                apod=synth.APOD_HANN, F=F)
    assert oracle.receive_weight(g, oracle.voxel_positions(g))[0, 0] == 0.0
    # a tilted element normal: rotating voxel and normal together keeps w
    th = math.radians(20)
    R = np.array([[math.cos(th), 0, math.sin(th)], [0, 1, 0], [-math.sin(th), 0, math.cos(th)]])
    v = R @ np.array([a / 2, 0, z])
    g = _single([0, 0, 0], v, synth.TX_NONE, [0, 0, 0], 0, 1540, 30e6, 0,
                apod=synth.APOD_HANN, F=F, normal=R @ np.array([0, 0, 1.0]))
    assert oracle.receive_weight(g, oracle.voxel_positions(g))[0, 0] == pytest.approx(0.5, abs=1e-12)


# ---------------------------------------------------------------------------
# Operator properties
# ---------------------------------------------------------------------------

def test_linearity():
    g = _small_geometry()
    rng = np.random.default_rng(0)
    y1 = rng.normal(size=(2, g.Q, g.M, g.K))
    y2 = rng.normal(size=(2, g.Q, g.M, g.K))
    a, b = 0.7, 1.9
    lhs = oracle.forward(a * y1 + b * y2, g)
    rhs = a * oracle.forward(y1, g) + b * oracle.forward(y2, g)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12 * np.abs(rhs).max())


def test_adjoint_dot_product():
    """<A y, x> = <y, A^T x> to 1e-12 (relative)."""
    g = _small_geometry()
    rng = np.random.default_rng(1)
    y = rng.normal(size=(2, g.Q, g.M, g.K))
    x = rng.normal(size=(2, g.N))
    wtx = rng.uniform(0.2, 1.0, size=(g.Q, g.N))
    lhs = np.sum(oracle.forward(y, g, w_tx=wtx) * x)
    rhs = np.sum(y * oracle.adjoint(x, g, w_tx=wtx))
    assert abs(lhs) > 1.0                      # not a cancellation to near zero
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_covers_out_of_range_taps():
    """cfg1 has taps past K; the dot test still holds there."""
    g = synth.cfg1()
    rng = np.random.default_rng(2)
    y = rng.normal(size=(1, g.Q, g.M, g.K))
    x = rng.normal(size=(1, g.N))
    f, _ = _f_and_w(g)
    assert (np.floor(f) + 1 >= g.K).mean() > 0.01
    lhs = np.sum(oracle.forward(y, g) * x)
    rhs = np.sum(y * oracle.adjoint(x, g))
    assert abs(lhs) > 1.0
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_translation_invariance():
    g = _small_geometry(kind=synth.TX_DIVERGING)
    g = g.replace(tx_kind=np.array([synth.TX_DIVERGING, synth.TX_NONE], np.int32))
    rng = np.random.default_rng(3)
    y = rng.normal(size=(1, g.Q, g.M, g.K))
    d = np.array([1.3e-3, -0.7e-3, 0.4e-3])
    gt = g.replace(elem_pos=g.elem_pos + d, tx_vec=g.tx_vec + d * np.array([[1], [0]]),
                   grid_origin=tuple(np.asarray(g.grid_origin) + d))
    np.testing.assert_allclose(oracle.forward(y, gt), oracle.forward(y, g), rtol=1e-10, atol=1e-10)


def test_receiver_permutation_invariance():
    g = _small_geometry()
    rng = np.random.default_rng(4)
    y = rng.normal(size=(1, g.Q, g.M, g.K))
    perm = rng.permutation(g.M)
    gp = g.replace(elem_pos=g.elem_pos[perm])
    np.testing.assert_allclose(oracle.forward(y[:, :, perm], gp), oracle.forward(y, g),
                               rtol=1e-13, atol=1e-12)


def test_mirror_symmetry():
    """Mirroring x -> -x of array, sources and grid mirrors the image."""
    g = synth.cfg2(dims=(6, 4, 3), n_side=4).replace(num_samples=600)
    rng = np.random.default_rng(5)
    y = rng.normal(size=(1, g.Q, g.M, g.K))
    nside = 4
    # element (i, j) -> (n-1-i, j); virtual source (a, b) -> (3-a, b)
    em = np.array([(nside - 1 - (m % nside)) + nside * (m // nside) for m in range(g.M)])
    qm = np.array([(3 - (q % 4)) + 4 * (q // 4) for q in range(g.Q)])
    ym = y[:, qm][:, :, em]
    x = oracle.forward(y, g)[0].reshape(3, 4, 6)
    xm = oracle.forward(ym, g)[0].reshape(3, 4, 6)
    np.testing.assert_allclose(xm, x[:, :, ::-1], rtol=1e-10, atol=1e-10)


def test_sound_speed_derivative_vs_finite_differences():
    """Central differences in c.  The interpolant is piecewise linear in f, so
    with a step too small for any tap index to change (checked) the difference
    quotient equals the analytic slope up to rounding; a coarse step that
    crosses many kinks of white-noise data still agrees to ~10%."""
    g = synth.cfg5()
    g = synth.sub_grid(g, (28, 28, 20), (4, 4, 4))
    rng = np.random.default_rng(6)
    y = rng.normal(size=(1, g.Q, g.M, g.K))
    d = oracle.dforward_dc(y, g)
    p = oracle.voxel_positions(g)
    path = oracle.transmit_path(g, p)[:, None, :] + oracle.receive_path(g, p)[None, :, :]
    for h, tol in ((2e-6, 1e-7), (0.1, 0.15)):
        if h < 1e-3:
            k_lo = np.floor(oracle.fractional_index(path, 0.0, g.c - h, g.fs, g.t0))
            k_hi = np.floor(oracle.fractional_index(path, 0.0, g.c + h, g.fs, g.t0))
            assert np.array_equal(k_lo, k_hi)
        fd = (oracle.forward(y, g, c=g.c + h) - oracle.forward(y, g, c=g.c - h)) / (2 * h)
        rel = np.linalg.norm(fd - d) / np.linalg.norm(d)
        assert rel < tol, (h, rel)


def test_sound_speed_derivative_fd_at_1e_3():
    """Central differences with h = 1e-3 m/s on a cfg5 sub-grid, data simulated
    at 1500 m/s.  x(c) is piecewise linear in each fractional index f, so the
    difference quotient equals the analytic (right-hand) slope for every term
    whose tap index stays put over [c - h, c + h]; a term whose f crosses an
    integer k_b adds at most |w| |s(k_b+1) - 2 s(k_b) + s(k_b-1)| |df/dc| (the
    jump of the slope at the kink).  Voxels without a crossing must agree to
    1e-7 relative; the others within the sum of those jumps."""
    g = synth.sub_grid(synth.cfg5(), (28, 28, 20), (4, 4, 4))
    _, _, y = synth.cfg5_data()
    y = y.numpy()[None].astype(np.float64)
    h = 1e-3
    d = oracle.dforward_dc(y, g)[0]
    fd = ((oracle.forward(y, g, c=g.c + h) - oracle.forward(y, g, c=g.c - h)) / (2 * h))[0]
    p = oracle.voxel_positions(g)
    path = oracle.transmit_path(g, p)[:, None, :] + oracle.receive_path(g, p)[None, :, :]
    f_lo = oracle.fractional_index(path, 0.0, g.c + h, g.fs, g.t0)      # f falls as c grows
    f_hi = oracle.fractional_index(path, 0.0, g.c - h, g.fs, g.t0)
    kb = np.floor(f_hi).astype(np.int64)
    cross = np.floor(f_lo) != kb                                        # [Q, M, N]
    assert cross.any() and not np.all(np.floor(f_hi) - np.floor(f_lo) <= 0)
    assert np.all(np.floor(f_hi) - np.floor(f_lo) <= 1)                 # one kink at most

    def s(j):
        K = g.K
        ok = (j >= 0) & (j < K)
        jc = np.clip(j, 0, K - 1)
        q = np.arange(g.Q)[:, None, None]
        m = np.arange(g.M)[None, :, None]
        return np.where(ok, y[0][q, m, jc], 0.0)

    jump = np.abs(s(kb + 1) - 2.0 * s(kb) + s(kb - 1))
    dfdc = g.fs * path / (g.c - h) ** 2                                 # >= |df/dc| on the interval
    bound = np.sum(np.where(cross, jump * dfdc, 0.0), axis=(0, 1))      # uniform weights: w = 1
    err = np.abs(fd - d)
    clean = bound == 0.0
    scale = np.abs(d).max()
    assert clean.any() and (~clean).any()
    assert np.all(err[clean] <= 1e-7 * scale)
    assert np.all(err[~clean] <= bound[~clean] * (1 + 1e-3) + 1e-7 * scale)


def test_slab_parallel_forward_equals_forward():
    """The process-pool evaluation used for timing is the same sum."""
    g = synth.cfg1()
    rng = np.random.default_rng(9)
    y = rng.normal(size=(2, g.Q, g.M, g.K))
    idx = np.sort(rng.choice(g.N, size=1500, replace=False))
    x1 = oracle.forward(y, g, voxels=idx)
    x2, used = oracle.forward_slabs_parallel(y, g, voxels=idx, workers=3, chunk=256)
    assert used == 3
    np.testing.assert_allclose(x2, x1, rtol=1e-14, atol=1e-14 * np.abs(x1).max())
    x3, _ = oracle.forward_slabs_parallel(y, g, workers=2, chunk=1000)
    np.testing.assert_allclose(x3, oracle.forward(y, g), rtol=1e-14, atol=1e-13)


def test_arithmetic_facts():
    """Sec. 2: N M Q time-of-flight evaluations and their FP32 storage."""
    N, M, Q = 128 ** 3, 32 ** 2, 16
    assert N * M * Q == 34_359_738_368
    assert N * M * Q * 4 == 128 * 2 ** 30

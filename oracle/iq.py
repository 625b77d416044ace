"""Complex baseband (IQ) delay-and-sum with phase rotation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's data model is complex baseband IQ (Sec. 2) while Eq. (2) carries
no phase term; beamforming demodulated data needs one.  Reading taken (the
standard baseband beamformer): the IQ record of a channel is its analytic RF
signal demodulated at the carrier fc, y_iq(t_k) = y_a(t_k) exp(-i 2 pi fc t_k)
with t_k = t0 + k/fs.  Each term is interpolated on the baseband samples at
the fractional index of Eq. (1) and remodulated with the two-way path time
tau = (D_tx + D_rx)/c:

    x[b, n] = sum_q sum_m w ((1 - alpha) s(k) + alpha s(k+1)) exp(i 2 pi fc tau),

which, for a slowly varying baseband, equals the analytic RF beamformer.
"""
from __future__ import annotations

import numpy as np

from .das import (_OneElement, _terms, fractional_index, receive_weight, sample,
                  voxel_positions)


def forward_iq(y_iq, g, fc: float, voxels=None, w_tx=None, c=None) -> np.ndarray:
    """y_iq: complex [B, Q, M, K] (or [Q, M, K]).  Returns complex128 [B, n]."""
    y = np.asarray(y_iq, np.complex128)
    if y.ndim == 3:
        y = y[None]
    B, Q, M, K = y.shape
    c = float(g.c if c is None else c)
    p = voxel_positions(g, voxels)
    d_tx, wt = _terms(g, p, c, w_tx)
    x = np.zeros((B, p.shape[0]), np.complex128)
    for m in range(M):
        d_rx = np.linalg.norm(p - np.asarray(g.elem_pos, np.float64)[m], axis=1)
        w_rx = receive_weight(_OneElement(g, m), p)[0]
        f = fractional_index(d_tx, d_rx[None, :], c, g.fs, g.t0)            # [Q, n]
        k = np.floor(f)
        alpha = f - k
        k = k.astype(np.int64)
        tau = (d_tx + d_rx[None, :]) / c                                     # [Q, n] seconds
        rot = np.exp(2j * np.pi * fc * tau)
        w = wt * w_rx[None, :]
        trace = y[:, :, m, :]
        s1 = sample(trace.real, k) + 1j * sample(trace.imag, k)
        s2 = sample(trace.real, k + 1) + 1j * sample(trace.imag, k + 1)
        x += np.sum((w * rot)[None] * ((1.0 - alpha[None]) * s1 + alpha[None] * s2), axis=1)
    return x


def adjoint_iq(gx, g, fc: float, w_tx=None, c=None) -> np.ndarray:
    """The transpose of ``forward_iq`` as a real-linear map on (Re, Im) lanes.

    forward_iq is complex-linear in y, so under the real inner product
    Re(sum a conj(b)) its transpose is the conjugate transpose: each tap of a
    term receives w conj(exp(i 2 pi fc tau)) times its interpolation weight
    times the upstream gradient,

        gy[b, q, m, j] = sum_n w exp(-i 2 pi fc tau) ((1-alpha)[j = k] + alpha [j = k+1]) gx[b, n],

    taps outside [0, K) dropped (they read zero in the forward map).  gx:
    complex [B, N] (or [N]) over the whole grid.  Returns complex128
    [B, Q, M, K]."""
    gx = np.asarray(gx, np.complex128)
    if gx.ndim == 1:
        gx = gx[None]
    B = gx.shape[0]
    Q, M, K = int(np.asarray(g.tx_kind).shape[0]), int(np.asarray(g.elem_pos).shape[0]), int(g.num_samples)
    c = float(g.c if c is None else c)
    p = voxel_positions(g)
    d_tx, wt = _terms(g, p, c, w_tx)
    gy = np.zeros((B, Q, M, K), np.complex128)
    for m in range(M):
        d_rx = np.linalg.norm(p - np.asarray(g.elem_pos, np.float64)[m], axis=1)
        w_rx = receive_weight(_OneElement(g, m), p)[0]
        f = fractional_index(d_tx, d_rx[None, :], c, g.fs, g.t0)
        k = np.floor(f)
        alpha = f - k
        k = k.astype(np.int64)
        tau = (d_tx + d_rx[None, :]) / c
        wr = wt * w_rx[None, :] * np.exp(-2j * np.pi * fc * tau)             # [Q, n]
        for b in range(B):
            for q in range(Q):
                for tap, cf in ((k[q], 1.0 - alpha[q]), (k[q] + 1, alpha[q])):
                    ok = (tap >= 0) & (tap < K)
                    v = wr[q] * cf * gx[b]
                    gy[b, q, m] += (np.bincount(tap[ok], weights=v[ok].real, minlength=K)
                                    + 1j * np.bincount(tap[ok], weights=v[ok].imag, minlength=K))
    return gy

def dforward_dc_iq(y_iq, g, fc: float, voxels=None, w_tx=None, c=None) -> np.ndarray:
    """d x[b, n] / d c of ``forward_iq``.  Both the fractional index and the
    phase depend on c through tau = (D_tx + D_rx)/c, dtau/dc = -tau/c:

        dx/dc = sum_q sum_m w exp(i 2 pi fc tau)
                ((s(k+1) - s(k)) df/dc + i 2 pi fc dtau/dc ((1-alpha) s(k) + alpha s(k+1))),

    with df/dc = fs dtau/dc (the right-hand slope at integer f, as for the
    real form, reading R8).  Returns complex128 [B, n]."""
    y = np.asarray(y_iq, np.complex128)
    if y.ndim == 3:
        y = y[None]
    B, Q, M, K = y.shape
    c = float(g.c if c is None else c)
    p = voxel_positions(g, voxels)
    d_tx, wt = _terms(g, p, c, w_tx)
    out = np.zeros((B, p.shape[0]), np.complex128)
    for m in range(M):
        d_rx = np.linalg.norm(p - np.asarray(g.elem_pos, np.float64)[m], axis=1)
        w_rx = receive_weight(_OneElement(g, m), p)[0]
        f = fractional_index(d_tx, d_rx[None, :], c, g.fs, g.t0)
        k = np.floor(f)
        alpha = f - k
        k = k.astype(np.int64)
        tau = (d_tx + d_rx[None, :]) / c
        dtau = -tau / c
        rot = np.exp(2j * np.pi * fc * tau)
        w = wt * w_rx[None, :]
        trace = y[:, :, m, :]
        s1 = sample(trace.real, k) + 1j * sample(trace.imag, k)
        s2 = sample(trace.real, k + 1) + 1j * sample(trace.imag, k + 1)
        interp = (1.0 - alpha[None]) * s1 + alpha[None] * s2
        slope = (s2 - s1) * (g.fs * dtau)[None]
        turn = 2j * np.pi * fc * dtau[None] * interp
        out += np.sum((w * rot)[None] * (slope + turn), axis=1)
    return out


def grad_sound_speed_iq(y_iq, gx, g, fc: float, w_tx=None, c=None) -> float:
    """dL/dc for a real loss of the complex image with upstream gradient
    gx = dL/dRe x + i dL/dIm x: sum_{b, n} Re(conj(gx) dx/dc)."""
    d = dforward_dc_iq(y_iq, g, fc, None, w_tx, c)
    return float(np.sum((np.conj(np.asarray(gx, np.complex128).reshape(d.shape)) * d).real))


def demodulate(y_analytic, fs: float, t0: float, fc: float) -> np.ndarray:
    """Analytic RF records [..., K] -> IQ baseband records (sample k at t0 + k/fs)."""
    K = np.asarray(y_analytic).shape[-1]
    t = t0 + np.arange(K) / fs
    return np.asarray(y_analytic, np.complex128) * np.exp(-2j * np.pi * fc * t)

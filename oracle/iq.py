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


def demodulate(y_analytic, fs: float, t0: float, fc: float) -> np.ndarray:
    """Analytic RF records [..., K] -> IQ baseband records (sample k at t0 + k/fs)."""
    K = np.asarray(y_analytic).shape[-1]
    t = t0 + np.arange(K) / fs
    return np.asarray(y_analytic, np.complex128) * np.exp(-2j * np.pi * fc * t)

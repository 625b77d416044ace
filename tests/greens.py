"""Frequency-domain point-scatterer simulator for the oracle's physical pins.

Follows the simulation model of Sec. 4.1: free-space Green's function
G(w; r, r') = exp(-i w |r - r'| / c) / |r - r'|, an incident field at each
scatterer, the scattered field summed at each receiver, and an inverse FFT to
time-domain samples.  The incident fields used here are an ideal plane wave
travelling along u (phase exp(-i w u.s / c)) and a point source at v
(G(w; v, s)).  Nothing here evaluates the beamformer's delay formula: the
echo times come out of the physics, and the tests compare them with the
oracle.
"""
from __future__ import annotations

import math

import numpy as np


def gaussian_pulse_spectrum(freqs, fc, sigma):
    """Spectrum of exp(-t^2 / 2 sigma^2) cos(2 pi fc t) (time origin at the
    envelope peak), Fourier convention Y(f) = int y(t) exp(-i 2 pi f t) dt."""
    a = sigma * math.sqrt(2.0 * math.pi) / 2.0
    return a * (np.exp(-2.0 * (math.pi * sigma * (freqs - fc)) ** 2)
                + np.exp(-2.0 * (math.pi * sigma * (freqs + fc)) ** 2))


def simulate(elem_pos, scat_pos, scat_amp, incident, c, fs, t0, K, fc, sigma, nfft=None,
             analytic_out=False):
    """Real channel data y[M, K] for one transmit (complex analytic record if
    analytic_out).  incident: ("plane", u) or ("point", v).  Samples at
    t0 + k/fs."""
    nfft = nfft or 4 * K
    freqs = np.fft.fftfreq(nfft, d=1.0 / fs)
    w = 2.0 * math.pi * freqs
    P = gaussian_pulse_spectrum(freqs, fc, sigma)
    Y = np.zeros((elem_pos.shape[0], nfft), np.complex128)
    for s, a in zip(np.atleast_2d(scat_pos), np.atleast_1d(scat_amp)):
        kind, vec = incident
        if kind == "plane":
            T = np.exp(-1j * w * (np.dot(vec, s) / c))
        else:
            d = np.linalg.norm(s - vec)
            T = np.exp(-1j * w * d / c) / d
        dr = np.linalg.norm(elem_pos - s, axis=1)                       # [M]
        G = np.exp(-1j * w[None, :] * dr[:, None] / c) / dr[:, None]
        Y += a * P[None, :] * G * T[None, :]
    # the record starts at t0: advance by t0
    Y *= np.exp(1j * w * t0)[None, :]
    if analytic_out:
        Y = Y * (2.0 * (freqs > 0) + 1.0 * (freqs == 0))[None, :]
        return np.fft.ifft(Y, axis=1)[:, :K] * fs
    y = np.fft.ifft(Y, axis=1).real * fs
    return y[:, :K]


def analytic(y):
    """Analytic signal along the last axis via the one-sided spectrum."""
    n = y.shape[-1]
    F = np.fft.fft(y, axis=-1)
    h = np.zeros(n)
    h[0] = 1.0
    if n % 2 == 0:
        h[n // 2] = 1.0
        h[1:n // 2] = 2.0
    else:
        h[1:(n + 1) // 2] = 2.0
    return np.fft.ifft(F * h, axis=-1)


def peak_time_samples(trace):
    """Envelope peak position in samples: 3-point parabola on log |analytic|
    (exact for a Gaussian envelope).  trace: real record or analytic record."""
    env = np.abs(trace) if np.iscomplexobj(trace) else np.abs(analytic(trace))
    i = int(np.argmax(env))
    l0, l1, l2 = np.log(env[i - 1]), np.log(env[i]), np.log(env[i + 1])
    return i + 0.5 * (l0 - l2) / (l0 - 2.0 * l1 + l2)

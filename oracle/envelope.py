"""Envelope of delay-and-sum volumes for the oracle (test infrastructure only).

The analytic channel data are y + i H{y} with H the discrete Hilbert
transform of the full record (scipy.signal.hilbert, FFT-based); beamforming
the real and imaginary parts as two batch lanes and taking the magnitude gives
the envelope (complex data ride the batch dimension, reading R6).
"""
import numpy as np
from scipy.signal import hilbert

from .das import forward


def analytic_lanes(y):
    """y[..., K] -> [2, ..., K] float64 (Re, Im) of the analytic signal."""
    z = hilbert(np.asarray(y, np.float64), axis=-1)
    return np.stack([z.real, z.imag])


def envelope(y, g, voxels=None, c=None):
    """|DAS(Re y~) + i DAS(Im y~)| for real channel data y[Q, M, K]."""
    lanes = analytic_lanes(y)
    x = forward(lanes, g, voxels=voxels, c=c)
    return np.hypot(x[0], x[1])


def envelope_energy(y, g, c=None, voxels=None):
    """sum_n |x~_n|^2."""
    lanes = analytic_lanes(y)
    x = forward(lanes, g, voxels=voxels, c=c)
    return float(np.sum(x[0] ** 2 + x[1] ** 2))


def focus_criterion(x_re, x_im):
    """The autofocus criterion of a complex volume: sum_n |x~_n|^4 / sum_n |x~_n|^2
    (energy-weighted mean intensity; unchanged by a pure magnification of a
    well-sampled image, largest when its echoes are best focused)."""
    e2 = np.asarray(x_re, np.float64) ** 2 + np.asarray(x_im, np.float64) ** 2
    return float(np.sum(e2 * e2) / np.sum(e2))

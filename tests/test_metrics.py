"""CPU checks of the envelope and image-quality helpers (product and oracle)."""
import math

import numpy as np
import pytest
import torch

from oracle import envelope as oenv
from paper_2606_13259_amd import metrics


def test_hilbert_of_cosine_is_sine():
    K = 512
    k = np.arange(K)
    y = np.cos(2 * np.pi * 8 * k / K)
    lanes = metrics.analytic_lanes(torch.from_numpy(y))
    np.testing.assert_allclose(lanes[0].numpy(), y, atol=1e-6)
    np.testing.assert_allclose(lanes[1].numpy(), np.sin(2 * np.pi * 8 * k / K), atol=1e-6)
    ol = oenv.analytic_lanes(y)
    np.testing.assert_allclose(ol[1], np.sin(2 * np.pi * 8 * k / K), atol=1e-12)


def test_point_target_peak_and_width_of_a_gaussian():
    # separable Gaussian blob: -6 dB full width = 2 sqrt(2 ln 2) sigma
    nx = ny = nz = 33
    sig = np.array([2.0, 3.0, 1.5])
    c = np.array([16.3, 15.6, 16.8])
    z, yy, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    v = np.exp(-0.5 * (((x - c[0]) / sig[0]) ** 2 + ((yy - c[1]) / sig[1]) ** 2
                       + ((z - c[2]) / sig[2]) ** 2))
    (pos, wid), = metrics.point_targets(torch.from_numpy(v), (0, 0, 0), (1, 1, 1), [c])
    np.testing.assert_allclose(pos, c, atol=0.08)
    np.testing.assert_allclose(wid, 2 * math.sqrt(2 * math.log(2)) * sig, rtol=0.03)


def test_envelope_db_error():
    r = torch.tensor([1.0, 0.5, 0.01, 1e-5], dtype=torch.float64)
    e = torch.tensor([1.0, 0.5 * 10 ** (0.1 / 20), 0.01, 5.0], dtype=torch.float64)
    mx, mean = metrics.envelope_db_error(e, r, floor_db=-40)
    assert mx == pytest.approx(0.1, abs=1e-9)       # the -100 dB voxel is excluded
    assert mean == pytest.approx(0.1 / 3, abs=1e-9)


def test_focus_criterion_is_magnification_invariant_and_peaks_at_focus():
    """sum e^4 / sum e^2 of a well-sampled Gaussian blob does not change when
    the blob is magnified (its widths scaled, peak kept), and falls when the
    blob is defocused (widths scaled with the energy kept, peak lowered)."""
    z, yy, x = np.meshgrid(np.arange(64), np.arange(64), np.arange(64), indexing="ij")

    def blob(sig, amp):
        e = amp * np.exp(-0.5 * (((x - 31.7) / sig[0]) ** 2 + ((yy - 32.2) / sig[1]) ** 2
                                 + ((z - 30.9) / sig[2]) ** 2))
        return np.sqrt(e), np.zeros_like(e)          # |x~|^2 = e

    sig = np.array([2.5, 3.0, 2.0])
    base = oenv.focus_criterion(*blob(sig, 1.0))
    assert base == pytest.approx(1.0 / 2 ** 1.5, rel=1e-6)     # exp^2 / exp over 3 Gaussians
    assert oenv.focus_criterion(*blob(1.3 * sig, 1.0)) == pytest.approx(base, rel=1e-6)
    # defocus: same energy spread over a 1.3x wider blob
    assert oenv.focus_criterion(*blob(1.3 * sig, 1.3 ** -3)) < 0.5 * base

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

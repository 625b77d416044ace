"""Pins of the SVD clutter filter / power Doppler oracle (CPU)."""
import numpy as np
import pytest

import synth
from oracle.clutter import casorati, power_doppler, svd_filter


def _known_svd(N=300, T=24, seed=0):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.normal(size=(N, T)))
    V, _ = np.linalg.qr(rng.normal(size=(T, T)))
    s = np.sort(rng.uniform(0.1, 10.0, T))[::-1] * np.logspace(2, 0, T)
    S = (U * s) @ V.T
    return S.T.copy(), U, s, V        # x[T, N]


@pytest.mark.parametrize("k_lo,k_hi", [(0, 24), (3, 24), (3, 20), (0, 1), (10, 11)])
def test_closed_form_on_a_known_decomposition(k_lo, k_hi):
    """x built from chosen orthonormal U, V and sigma: the oracle returns that
    sigma and P[n] = (1/T) sum_{j kept} sigma_j^2 U[n, j]^2."""
    x, U, s, V = _known_svd()
    sig, P = power_doppler(x, k_lo, k_hi)
    assert np.allclose(sig, s, rtol=1e-12, atol=0)
    keep = slice(k_lo, k_hi)
    P_ref = (U[:, keep] ** 2 * s[keep] ** 2).sum(1) / x.shape[0]
    assert np.allclose(P, P_ref, rtol=1e-9, atol=1e-12 * P_ref.max())


def test_keeping_everything_is_the_identity():
    x = synth.doppler_ensemble((8, 6, 5), T=20, seed=1)[0]
    sig, xf = svd_filter(x, 0, 20)
    assert np.allclose(xf, x, rtol=0, atol=1e-10 * np.abs(x).max())
    assert np.allclose(power_doppler(x, 0, 20)[1], np.mean(x.astype(np.float64) ** 2, 0), rtol=1e-10)


def test_singular_values_by_an_independent_route():
    """sigma^2 equals the eigenvalues of S^T S (symmetric eigensolver)."""
    x = synth.doppler_ensemble((8, 6, 5), T=32, seed=2)[0]
    S = casorati(x)
    lam = np.sort(np.linalg.eigvalsh(S.T @ S))[::-1]
    sig = power_doppler(x, 3, 32)[0]
    assert np.allclose(sig ** 2, lam, rtol=1e-9, atol=1e-9 * lam[0])


def test_filtered_signal_is_orthogonal_to_removed_components():
    x = synth.doppler_ensemble((8, 6, 5), T=32, seed=3)[0]
    S = casorati(x)
    _, _, Vt = np.linalg.svd(S, full_matrices=False)
    _, xf = svd_filter(x, 3, 30)
    Sf = casorati(xf)
    removed = np.concatenate([Vt[:3], Vt[30:]])
    assert np.abs(Sf @ removed.T).max() <= 1e-10 * np.abs(S).max() * np.sqrt(S.shape[0])


def test_component_bands_add_up():
    x = synth.doppler_ensemble((8, 6, 5), T=32, seed=4)[0]
    a = svd_filter(x, 2, 10)[1] + svd_filter(x, 10, 25)[1]
    assert np.allclose(a, svd_filter(x, 2, 25)[1], rtol=0, atol=1e-10 * np.abs(x).max())


def test_clutter_removal_on_the_synthetic_ensemble():
    """Removing the 3 clutter components leaves the vessel bright and the
    tissue at the noise floor (clutter is 40 dB above blood)."""
    x, vessel = synth.doppler_ensemble((16, 12, 8), T=48, seed=5)
    sig, P = power_doppler(x, 3, 48)
    assert sig[2] / sig[3] > 5.0             # a clear gap after the clutter rank
    assert np.median(P[vessel]) > 20 * np.median(P[~vessel])
    raw = np.mean(x.astype(np.float64) ** 2, 0)
    assert np.median(raw[~vessel]) > 1e3 * np.median(P[~vessel])

"""Rank-truncation (SVD) clutter filter and power Doppler of a beamformed ensemble.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper lists GPU rank truncation for clutter filtering among the
primitives that accompany its beamformer (Sec. 1, Sec. 5), without a formula.
Reading taken (the standard Casorati-matrix filter of ultrafast Doppler):

* the ensemble x[t][n] (T frames of N voxels) is arranged as the Casorati
  matrix S[n][t] = x[t][n] (N x T);
* S = U diag(sigma) V^T (thin SVD, sigma descending);
* the filter keeps the singular components k_lo .. k_hi-1: tissue clutter
  (the k_lo largest, slowly varying and spatially coherent) and, with
  k_hi < T, the noise tail are removed:
      S_f = sum_{k_lo <= j < k_hi} sigma_j u_j v_j^T;
* power Doppler is the mean filtered power per voxel:
      P[n] = (1/T) sum_t S_f[n][t]^2.

The SVD is the library routine (numpy, FP64) used as one step.
"""
from __future__ import annotations

import numpy as np


def casorati(x: np.ndarray) -> np.ndarray:
    """x[T, N] (frames of a volume, any trailing shape flattened) -> S[N, T] float64."""
    x = np.asarray(x, np.float64)
    return x.reshape(x.shape[0], -1).T


def svd_filter(x: np.ndarray, k_lo: int, k_hi: int):
    """(sigma[T], filtered ensemble xf[T, N]) keeping components k_lo .. k_hi-1."""
    S = casorati(x)
    T = S.shape[1]
    assert 0 <= k_lo < k_hi <= T
    U, s, Vt = np.linalg.svd(S, full_matrices=False)
    keep = slice(k_lo, k_hi)
    Sf = (U[:, keep] * s[keep]) @ Vt[keep]
    return s, Sf.T


def power_doppler(x: np.ndarray, k_lo: int, k_hi: int):
    """(sigma[T], P[N]) with P[n] = mean over frames of the filtered signal squared."""
    s, xf = svd_filter(x, k_lo, k_hi)
    return s, np.mean(xf ** 2, axis=0)

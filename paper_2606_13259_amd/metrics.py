"""Image-quality measures for delay-and-sum volumes (torch, CPU or GPU).

* ``analytic_lanes``: the analytic channel data y + i H{y} (FFT-based discrete
  Hilbert transform over the full K record), returned as two real batch lanes
  (Re, Im) so that one beamforming call images both (complex data ride the
  batch dimension).
* ``envelope``: |DAS(Re) + i DAS(Im)|.
* ``rel_l2``, ``envelope_db_error`` (dB error of an envelope against a
  reference envelope, over voxels within ``floor_db`` of the reference peak;
  envelopes are shown on a dB scale relative to their peak, Sec. 4.5 shows
  32 dB), ``point_targets`` (sub-voxel peak by 3-point parabolic fit and
  -6 dB widths along x, y, z around each target).
"""
from __future__ import annotations

import math

import numpy as np
import torch


def analytic_lanes(y: torch.Tensor) -> torch.Tensor:
    """y[..., K] real -> [2, ..., K]: (y, H{y}) with H the discrete Hilbert
    transform (one-sided spectrum, DC and Nyquist kept once)."""
    K = y.shape[-1]
    Y = torch.fft.fft(y.to(torch.float64), dim=-1)
    h = torch.zeros(K, dtype=torch.float64, device=y.device)
    h[0] = 1.0
    if K % 2 == 0:
        h[K // 2] = 1.0
        h[1:K // 2] = 2.0
    else:
        h[1:(K + 1) // 2] = 2.0
    za = torch.fft.ifft(Y * h, dim=-1)
    return torch.stack([za.real, za.imag]).to(torch.float32)


def envelope(x_re: torch.Tensor, x_im: torch.Tensor) -> torch.Tensor:
    return torch.sqrt(x_re.double() ** 2 + x_im.double() ** 2)


def rel_l2(x, x_ref) -> float:
    x = torch.as_tensor(x).double()
    r = torch.as_tensor(x_ref).double().to(x.device)
    return float(torch.linalg.norm(x - r) / torch.linalg.norm(r))


def envelope_db_error(env, env_ref, floor_db: float = -40.0):
    """(max, mean) of |20 log10(env/max env_ref) - 20 log10(env_ref/max env_ref)|
    over voxels where the reference is within floor_db of its peak."""
    e = torch.as_tensor(env).double().flatten()
    r = torch.as_tensor(env_ref).double().flatten().to(e.device)
    peak = r.max()
    keep = 20.0 * torch.log10(r / peak) >= floor_db
    d = (20.0 * torch.log10(e[keep] / peak) - 20.0 * torch.log10(r[keep] / peak)).abs()
    return float(d.max()), float(d.mean())


def _parabolic(v_m, v_0, v_p):
    den = v_m - 2.0 * v_0 + v_p
    return 0.0 if den == 0 else 0.5 * (v_m - v_p) / den


def _width_6db(line: np.ndarray, i0: int) -> float:
    """-6 dB full width (in samples) of a 1-D profile around its peak i0,
    by linear interpolation of the half-amplitude crossings."""
    half = line[i0] * 0.5
    left = i0
    while left > 0 and line[left] > half:
        left -= 1
    right = i0
    while right < len(line) - 1 and line[right] > half:
        right += 1
    if line[left] > half or line[right] > half:
        return float("nan")
    xl = left + (half - line[left]) / (line[left + 1] - line[left])
    xr = right - 1 + (line[right - 1] - half) / (line[right - 1] - line[right])
    return float(xr - xl)


def point_targets(env_vol, grid_origin, grid_spacing, targets, search: int = 3):
    """Per target: (peak position (m) from a 3-point parabolic fit along each
    axis around the envelope maximum within +-search voxels of the target's
    nearest voxel, -6 dB widths (m) along x, y, z).  env_vol: [Nz, Ny, Nx]."""
    v = np.asarray(torch.as_tensor(env_vol).double().cpu())
    nz, ny, nx = v.shape
    o = np.asarray(grid_origin, float)
    s = np.asarray(grid_spacing, float)
    out = []
    for t in np.atleast_2d(targets):
        c = np.rint((np.asarray(t) - o) / s).astype(int)  # (ix, iy, iz)
        lo = np.maximum(c - search, 0)
        hi = np.minimum(c + search + 1, [nx, ny, nz])
        if np.any(hi <= lo):
            out.append((np.full(3, np.nan), np.full(3, np.nan)))
            continue
        blk = v[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        kz, ky, kx = np.unravel_index(int(np.argmax(blk)), blk.shape)
        iz, iy, ix = lo[2] + kz, lo[1] + ky, lo[0] + kx
        pos = np.zeros(3)
        wid = np.zeros(3)
        for ax, (i, n, line) in enumerate(((ix, nx, v[iz, iy, :]), (iy, ny, v[iz, :, ix]),
                                           (iz, nz, v[:, iy, ix]))):
            d = _parabolic(line[i - 1], line[i], line[i + 1]) if 0 < i < n - 1 else 0.0
            pos[ax] = o[ax] + (i + d) * s[ax]
            wid[ax] = _width_6db(line, i) * s[ax]
        out.append((pos, wid))
    return out

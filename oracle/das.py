"""Plain FP64 NumPy definition of 3D delay-and-sum (forward, adjoint, d/dc).

TEST INFRASTRUCTURE ONLY: used by tests, the smoke check and the benchmark's
CPU-baseline leg, never by the product path.  Slow on purpose: one loop over
receivers, vectorised over voxels, observations and batch items, with no
blocking, tiling or reordering of the sum.

What is computed (paper, Sec. 2):

* Eq. (1): the time of flight splits into a transmit part and a receive part,
  tau = tau_tx + |p_n - r_m| / c0.  The transmit part follows the footnote to
  Eq. (1): a plane wave or a diverging wave from a virtual source; a
  photoacoustic acquisition has none.
* The weight is w = w_tx[q, n] * w_rx[m, n] (the paragraph after Eq. (1));
  w_tx is an optional precomputed [Q, N] table, w_rx is a function of the
  voxel and of the element's origin and direction.
* Eq. (2): x[n] = sum_q sum_m w * y_qm[tau], with linear interpolation between
  samples k = floor(tau) and k + 1 (the sentence after Eq. (2)).
* Channel data are batched as y[B, Q, M, K] (Sec. 2, last paragraphs); one
  output volume per batch item.

Readings of what the paper leaves open:

* R1 plane-wave sign: the descriptor is the propagation direction u (into the
  medium) and the transmit path is u.p, i.e. time zero is when the wavefront
  crosses the coordinate origin.  This is the footnote's form with d = -u.
* R2 time origins: every transmit carries a path offset L_q (metres) that is
  subtracted from its transmit path (default 0, which is the footnote's literal
  diverging-wave form: time zero at virtual emission); sample k of a channel is
  taken at t0 + k/fs, k = 0 .. K-1 (0-based; the text counts from 1).
* R3 fractional index: f = ((D_tx + D_rx)/c - t0) * fs in samples, with
  D_tx, D_rx path lengths in metres; k = floor(f), alpha = f - k.
* R4 out-of-range taps read zero: s(j) = y[j] for 0 <= j < K, else 0.
* R5 receive weight: uniform (1) or Hann with f-number F: with d = p - r_m,
  z = d.n_m, rho = |d - z n_m|, a = z / (2F):
  w_rx = (1 + cos(pi rho / a)) / 2 when z > 0 and rho < a, else 0.
* R6 real data; complex data are two real batch lanes (Re, Im).
* R7 adjoint: the exact transpose of the forward map y -> x above.
* R8 sound-speed derivative: grid and w_rx do not depend on c; t0 is a time;
  d f / d c = -fs (D_tx + D_rx) / c^2; at integer f the right-hand slope
  s(k+1) - s(k) is used (consistent with k = floor(f)).
* R15 higher-order interpolation (the paper allows other schemes after
  Eq. (2)): ``interp="cubic"`` is the four-point Lagrange interpolant through
  samples k-1, k, k+1, k+2 (k = floor(f), alpha = f - k), which reproduces
  every cubic polynomial; taps outside [0, K) read zero as in R4.
"""
from __future__ import annotations

import math
import os

import numpy as np

TX_NONE, TX_PLANE, TX_DIVERGING = 0, 1, 2
APOD_UNIFORM, APOD_HANN = 0, 1

__all__ = [
    "TX_NONE", "TX_PLANE", "TX_DIVERGING", "APOD_UNIFORM", "APOD_HANN",
    "voxel_positions", "transmit_path", "receive_path", "receive_weight",
    "fractional_index", "sample", "tap_weights", "forward", "adjoint", "dforward_dc",
    "grad_sound_speed", "nonzero_counts", "forward_slabs_parallel",
]


def _normals(g, M):
    n = getattr(g, "elem_normal", None)
    if n is None:
        out = np.zeros((M, 3))
        out[:, 2] = 1.0
        return out
    n = np.asarray(n, np.float64)
    return n / np.linalg.norm(n, axis=1, keepdims=True)


def voxel_positions(g, idx=None) -> np.ndarray:
    """p_n for the voxel grid (Sec. 2), n = ix + Nx (iy + Ny iz); [n, 3]."""
    nx, ny, nz = (int(v) for v in g.grid_dims)
    n = np.arange(nx * ny * nz) if idx is None else np.asarray(idx, np.int64)
    ix = n % nx
    iy = (n // nx) % ny
    iz = n // (nx * ny)
    o = np.asarray(g.grid_origin, np.float64)
    s = np.asarray(g.grid_spacing, np.float64)
    return o + np.stack([ix, iy, iz], axis=-1).astype(np.float64) * s


def transmit_path(g, p) -> np.ndarray:
    """c0 * tau_tx for every transmit and voxel, [Q, n] metres.

    Footnote to Eq. (1), with readings R1 and R2."""
    kinds = np.asarray(g.tx_kind)
    vecs = np.asarray(g.tx_vec, np.float64)
    offs = np.asarray(g.tx_offset, np.float64)
    out = np.zeros((kinds.shape[0], p.shape[0]))
    for q, kind in enumerate(kinds):
        if kind == TX_PLANE:
            out[q] = p @ vecs[q]
        elif kind == TX_DIVERGING:
            out[q] = np.linalg.norm(p - vecs[q], axis=1)
        elif kind == TX_NONE:
            out[q] = 0.0
        else:
            raise ValueError(f"unknown transmit kind {kind}")
        out[q] -= offs[q]
    return out


def receive_path(g, p) -> np.ndarray:
    """c0 * tau_rx = |p_n - r_m|, [M, n] metres (Eq. (1))."""
    r = np.asarray(g.elem_pos, np.float64)
    return np.linalg.norm(p[None, :, :] - r[:, None, :], axis=2)


def receive_weight(g, p) -> np.ndarray:
    """w_rx[m, n] (reading R5), [M, n]."""
    r = np.asarray(g.elem_pos, np.float64)
    M = r.shape[0]
    if int(g.apod) == APOD_UNIFORM:
        return np.ones((M, p.shape[0]))
    if int(g.apod) != APOD_HANN:
        raise ValueError(f"unknown apodization {g.apod}")
    nrm = _normals(g, M)
    F = float(g.f_number)
    d = p[None, :, :] - r[:, None, :]                       # [M, n, 3]
    z = np.einsum("mnk,mk->mn", d, nrm)
    lateral = d - z[..., None] * nrm[:, None, :]
    rho = np.linalg.norm(lateral, axis=2)
    a = z / (2.0 * F)
    inside = (z > 0) & (rho < a)
    w = np.zeros_like(z)
    w[inside] = 0.5 * (1.0 + np.cos(np.pi * rho[inside] / a[inside]))
    return w


def fractional_index(d_tx, d_rx, c, fs, t0):
    """f = ((D_tx + D_rx)/c - t0) * fs (Eq. (1) with reading R3)."""
    return ((d_tx + d_rx) / c - t0) * fs


def sample(trace, j):
    """s(j) (reading R4): trace [B, Q, K], integer taps j [Q, n] -> [B, Q, n].

    Returns trace[b, q, j[q, n]] where 0 <= j < K and 0 elsewhere."""
    K = trace.shape[-1]
    inside = (j >= 0) & (j < K)
    jc = np.clip(j, 0, K - 1)
    q = np.arange(trace.shape[1])[:, None]
    return np.where(inside[None], trace[:, q, jc], 0.0)


def tap_weights(alpha, interp="linear"):
    """[(offset, weight)] of the interpolant at fractional position alpha in
    [0, 1) after sample k: linear (the sentence after Eq. (2)) or the
    four-point Lagrange cubic (reading R15)."""
    a = alpha
    if interp == "linear":
        return [(0, 1.0 - a), (1, a)]
    if interp == "cubic":
        return [(-1, -a * (a - 1.0) * (a - 2.0) / 6.0),
                (0, (a + 1.0) * (a - 1.0) * (a - 2.0) / 2.0),
                (1, -(a + 1.0) * a * (a - 2.0) / 2.0),
                (2, (a + 1.0) * a * (a - 1.0) / 6.0)]
    raise ValueError(f"unknown interpolation {interp!r}")


def _terms(g, p, c, w_tx):
    """Per-voxel transmit paths and transmit weights."""
    d_tx = transmit_path(g, p)                                 # [Q, n]
    Q = d_tx.shape[0]
    wt = np.ones_like(d_tx) if w_tx is None else np.asarray(w_tx, np.float64).reshape(Q, -1)
    return d_tx, wt


def forward(y, g, voxels=None, w_tx=None, c=None, interp="linear") -> np.ndarray:
    """x[b, n] = sum_q sum_m w_qmn ((1-alpha) s(k) + alpha s(k+1)) (Eq. (2)).

    y: [B, Q, M, K] (any real dtype; promoted to float64).
    voxels: optional voxel indices (to evaluate a sample of the volume).
    w_tx: optional [Q, n] transmit weights for exactly those voxels.
    interp: "linear" (Eq. (2)) or "cubic" (reading R15: the sum of the
    four Lagrange tap weights times s(k-1) .. s(k+2)).
    Returns float64 [B, n]."""
    y = np.asarray(y, np.float64)
    if y.ndim == 3:
        y = y[None]
    B, Q, M, K = y.shape
    c = float(g.c if c is None else c)
    p = voxel_positions(g, voxels)
    d_tx, wt = _terms(g, p, c, w_tx)
    x = np.zeros((B, p.shape[0]))
    for m in range(M):
        d_rx = np.linalg.norm(p - np.asarray(g.elem_pos, np.float64)[m], axis=1)   # [n]
        w_rx = receive_weight(_OneElement(g, m), p)[0]                              # [n]
        f = fractional_index(d_tx, d_rx[None, :], c, g.fs, g.t0)                    # [Q, n]
        k = np.floor(f)
        alpha = f - k
        k = k.astype(np.int64)
        w = wt * w_rx[None, :]                                                      # [Q, n]
        trace = y[:, :, m, :]                                                       # [B, Q, K]
        if interp == "linear":
            s1 = sample(trace, k)                                                   # [B, Q, n]
            s2 = sample(trace, k + 1)
            x += np.sum(w[None] * ((1.0 - alpha[None]) * s1 + alpha[None] * s2), axis=1)
        else:
            v = np.zeros((B, Q, p.shape[0]))
            for off, coef in tap_weights(alpha, interp):
                v += coef[None] * sample(trace, k + off)
            x += np.sum(w[None] * v, axis=1)
    return x


class _OneElement:
    """View of a geometry restricted to element m (for the weight function)."""

    def __init__(self, g, m):
        self.elem_pos = np.asarray(g.elem_pos, np.float64)[m:m + 1]
        n = getattr(g, "elem_normal", None)
        self.elem_normal = None if n is None else np.asarray(n, np.float64)[m:m + 1]
        self.apod = g.apod
        self.f_number = g.f_number


def adjoint(gx, g, w_tx=None, c=None, interp="linear") -> np.ndarray:
    """gy[b, q, m, j] = sum_n w ((1-alpha)[j = k] + alpha [j = k+1]) gx[b, n].

    The exact transpose of ``forward`` (reading R7); taps outside [0, K) are
    dropped, as they read zero in the forward map.  gx: [B, N] over the whole
    grid.  With interp="cubic" the four Lagrange taps of reading R15 are
    scattered instead.  Returns float64 [B, Q, M, K]."""
    gx = np.asarray(gx, np.float64)
    if gx.ndim == 1:
        gx = gx[None]
    B = gx.shape[0]
    Q, M, K = int(np.asarray(g.tx_kind).shape[0]), int(np.asarray(g.elem_pos).shape[0]), int(g.num_samples)
    c = float(g.c if c is None else c)
    p = voxel_positions(g)
    d_tx, wt = _terms(g, p, c, w_tx)
    gy = np.zeros((B, Q, M, K))
    for m in range(M):
        d_rx = np.linalg.norm(p - np.asarray(g.elem_pos, np.float64)[m], axis=1)
        w_rx = receive_weight(_OneElement(g, m), p)[0]
        f = fractional_index(d_tx, d_rx[None, :], c, g.fs, g.t0)
        k = np.floor(f)
        alpha = f - k
        k = k.astype(np.int64)
        w = wt * w_rx[None, :]
        for b in range(B):
            for q in range(Q):
                for off, cf in tap_weights(alpha[q], interp):
                    tap, coef = k[q] + off, w[q] * cf
                    ok = (tap >= 0) & (tap < K)
                    gy[b, q, m] += np.bincount(tap[ok], weights=coef[ok] * gx[b, ok], minlength=K)
    return gy


def dforward_dc(y, g, voxels=None, w_tx=None, c=None) -> np.ndarray:
    """d x[b, n] / d c (reading R8): sum_q sum_m w (s(k+1) - s(k)) df/dc,
    with df/dc = -fs (D_tx + D_rx) / c^2.  Returns float64 [B, n]."""
    y = np.asarray(y, np.float64)
    if y.ndim == 3:
        y = y[None]
    B, Q, M, K = y.shape
    c = float(g.c if c is None else c)
    p = voxel_positions(g, voxels)
    d_tx, wt = _terms(g, p, c, w_tx)
    out = np.zeros((B, p.shape[0]))
    for m in range(M):
        d_rx = np.linalg.norm(p - np.asarray(g.elem_pos, np.float64)[m], axis=1)
        w_rx = receive_weight(_OneElement(g, m), p)[0]
        path = d_tx + d_rx[None, :]
        f = fractional_index(d_tx, d_rx[None, :], c, g.fs, g.t0)
        k = np.floor(f).astype(np.int64)
        dfdc = -g.fs * path / (c * c)
        w = wt * w_rx[None, :]
        trace = y[:, :, m, :]
        s1 = sample(trace, k)
        s2 = sample(trace, k + 1)
        out += np.sum(w[None] * (s2 - s1) * dfdc[None], axis=1)
    return out


def grad_sound_speed(y, gx, g, w_tx=None, c=None) -> float:
    """dL/dc = sum_{b, n} gx[b, n] d x[b, n]/d c for an upstream gradient gx."""
    d = dforward_dc(y, g, None, w_tx, c)
    return float(np.sum(np.asarray(gx, np.float64).reshape(d.shape) * d))


def nonzero_counts(g, voxels=None):
    """(P_nz, T_nz): numbers of (voxel, element) pairs and (voxel, element,
    transmit) triples with a nonzero receive weight (transmit weights of 1)."""
    p = voxel_positions(g, voxels)
    M = int(np.asarray(g.elem_pos).shape[0])
    Q = int(np.asarray(g.tx_kind).shape[0])
    pnz = 0
    for m in range(M):
        pnz += int(np.count_nonzero(receive_weight(_OneElement(g, m), p)[0]))
    return pnz, pnz * Q


# --------------------------------------------------------------------------
# whole-volume evaluation on all host cores (for timing the oracle)
# --------------------------------------------------------------------------

_POOL_STATE = {}


def _slab_worker(args):
    idx = args
    y, g = _POOL_STATE["y"], _POOL_STATE["g"]
    return forward(y, g, voxels=idx)


def _init_pool(y, g):
    _POOL_STATE["y"] = y
    _POOL_STATE["g"] = g


def forward_slabs_parallel(y, g, voxels=None, workers=None, chunk=4096):
    """``forward`` over ``voxels`` (default: all), split in chunks of voxels
    evaluated by a process pool.  Returns (x [B, n], workers used)."""
    import multiprocessing as mp
    nx, ny, nz = (int(v) for v in g.grid_dims)
    idx = np.arange(nx * ny * nz) if voxels is None else np.asarray(voxels, np.int64)
    workers = workers or os.cpu_count() or 1
    chunks = [idx[i:i + chunk] for i in range(0, idx.shape[0], chunk)]
    if workers == 1 or len(chunks) == 1:
        return forward(y, g, voxels=idx), 1
    ctx = mp.get_context("fork")
    with ctx.Pool(workers, initializer=_init_pool, initargs=(np.asarray(y, np.float64), g)) as pool:
        parts = pool.map(_slab_worker, chunks)
    return np.concatenate(parts, axis=1), workers

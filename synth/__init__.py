"""Seeded synthetic inputs for the 3D delay-and-sum path.

This module is shared by the tests, the benchmark and the smoke check.  It
builds geometries (array, transmits, voxel grid) for the five workloads the
method is measured on and synthesises channel data from point scatterers.  It
holds no part of the beamformer: no delay formation for voxels, no
interpolation, no weighting or summation over elements.  Both the FP64 oracle
and the HIP path receive the arrays made here and nothing else.

Workloads (sizes follow the problem statement of Sec. 2 and the evaluation
setup of Sec. 4.1; every reading the paper leaves open is stated here):

* ``cfg1``  8x8 array, pitch 0.2 mm, one 0-degree plane wave, K = 256,
  16^3 voxels at lambda/2 from z = 5 mm, uniform apodization, 3 scatterers
  plus N(0, 0.01) noise.
* ``cfg2``  32x32 array, pitch 0.3 mm, 16 diverging waves from a 4x4 grid of
  virtual sources 10 mm behind the array, K = 2048, 128^3 voxels at lambda/2,
  Hann receive apodization with f-number 1.5, 200 targets in speckle.
* ``cfg5``  16x16 array, pitch 0.3 mm, 8 steered plane waves, K = 1024,
  64^3 voxels, data made at c = 1500 m/s (the sound-speed autofocus case).
* ``cfg4``  ensembles of cfg2-geometry frames with seeded sub-wavelength
  motion, and mixed grids / array sizes.

Geometry conventions (the reading used throughout):

* voxel n = ix + Nx*(iy + Ny*iz) sits at origin + (ix, iy, iz) * spacing;
* element m = i + n_side*j sits at ((i-(n-1)/2) pitch, (j-(n-1)/2) pitch, 0),
  facing +z;
* a plane-wave descriptor holds the unit propagation direction u (into the
  medium); the transmit path is u.p - L;
* a diverging-wave descriptor holds the virtual source v; the transmit path is
  |p - v| - L;
* sample k of every channel is taken at time t0 + k/fs.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

TX_NONE, TX_PLANE, TX_DIVERGING = 0, 1, 2
APOD_UNIFORM, APOD_HANN = 0, 1

C_NOMINAL = 1540.0      # m/s
FC = 7.5e6              # Hz, carrier of every workload
FS = 30e6               # Hz
BANDWIDTH = 0.6         # -6 dB fractional bandwidth of the pulse


@dataclasses.dataclass
class Geometry:
    """Everything the beamformer needs apart from the channel data."""

    elem_pos: np.ndarray                 # [M, 3] float64, metres
    elem_normal: Optional[np.ndarray]    # [M, 3] float64 or None (= +z)
    tx_kind: np.ndarray                  # [Q] int32
    tx_vec: np.ndarray                   # [Q, 3] float64
    tx_offset: np.ndarray                # [Q] float64, metres
    grid_origin: tuple                   # (x0, y0, z0) metres
    grid_spacing: tuple                  # (dx, dy, dz) metres
    grid_dims: tuple                     # (Nx, Ny, Nz)
    num_samples: int                     # K
    c: float                             # m/s
    fs: float                            # Hz
    t0: float = 0.0                      # s
    apod: int = APOD_UNIFORM
    f_number: float = 1.0

    @property
    def M(self) -> int:
        return int(self.elem_pos.shape[0])

    @property
    def Q(self) -> int:
        return int(self.tx_kind.shape[0])

    @property
    def N(self) -> int:
        nx, ny, nz = self.grid_dims
        return int(nx * ny * nz)

    @property
    def K(self) -> int:
        return int(self.num_samples)

    def replace(self, **kw) -> "Geometry":
        return dataclasses.replace(self, **kw)

    def voxel_box(self):
        """(lo, hi) corners of the voxel-centre bounding box."""
        o = np.asarray(self.grid_origin, float)
        s = np.asarray(self.grid_spacing, float)
        d = np.asarray(self.grid_dims, float) - 1.0
        return o, o + d * s


def matrix_array(n_side: int, pitch: float) -> np.ndarray:
    """Element centres of an n_side x n_side matrix array in the z = 0 plane."""
    i = np.arange(n_side, dtype=np.float64) - (n_side - 1) / 2.0
    ex, ey = np.meshgrid(i * pitch, i * pitch, indexing="xy")   # m = i + n*j
    return np.stack([ex.ravel(), ey.ravel(), np.zeros(n_side * n_side)], axis=1)


def centred_grid(dims, spacing: float, z0: float):
    nx, ny, _ = dims
    origin = (-(nx - 1) / 2.0 * spacing, -(ny - 1) / 2.0 * spacing, z0)
    return origin, (spacing, spacing, spacing)


def plane_wave(theta_x_deg: float, theta_y_deg: float):
    sx = math.sin(math.radians(theta_x_deg))
    sy = math.sin(math.radians(theta_y_deg))
    return np.array([sx, sy, math.sqrt(1.0 - sx * sx - sy * sy)])


def _make_geometry(n_side, pitch, tx_kind, tx_vec, dims, K, apod, fnum,
                   c=C_NOMINAL, z0=5e-3, spacing=None):
    lam = C_NOMINAL / FC
    spacing = lam / 2.0 if spacing is None else spacing
    origin, sp = centred_grid(dims, spacing, z0)
    Q = len(tx_kind)
    return Geometry(
        elem_pos=matrix_array(n_side, pitch), elem_normal=None,
        tx_kind=np.asarray(tx_kind, np.int32),
        tx_vec=np.asarray(tx_vec, np.float64).reshape(Q, 3),
        tx_offset=np.zeros(Q), grid_origin=origin, grid_spacing=sp,
        grid_dims=tuple(int(d) for d in dims), num_samples=int(K), c=float(c),
        fs=FS, t0=0.0, apod=apod, f_number=float(fnum))


def cfg1() -> Geometry:
    """Tiny plain-FP32 case: 8x8 array, one 0-degree plane wave, 16^3 voxels."""
    return _make_geometry(8, 0.2e-3, [TX_PLANE], [plane_wave(0, 0)], (16, 16, 16),
                          256, APOD_UNIFORM, 1.0)


def diverging_sources() -> np.ndarray:
    """4x4 virtual sources 10 mm behind the array, q = a + 4b."""
    s = np.array([-3.6e-3, -1.2e-3, 1.2e-3, 3.6e-3])
    vx, vy = np.meshgrid(s, s, indexing="xy")
    return np.stack([vx.ravel(), vy.ravel(), np.full(16, -10e-3)], axis=1)


def cfg2(dims=(128, 128, 128), n_side=32) -> Geometry:
    """Full-scale case: 32x32 array, 16 diverging waves, 128^3 voxels, Hann F=1.5."""
    v = diverging_sources()
    return _make_geometry(n_side, 0.3e-3, [TX_DIVERGING] * 16, v, dims, 2048,
                          APOD_HANN, 1.5)


def cfg5(c=C_NOMINAL) -> Geometry:
    """Differentiable case: 16x16 array, 8 steered plane waves, 64^3 voxels."""
    angles = [(tx, ty) for ty in (-2.0, 2.0) for tx in (-4.5, -1.5, 1.5, 4.5)]
    vecs = [plane_wave(a, b) for a, b in angles]
    return _make_geometry(16, 0.3e-3, [TX_PLANE] * 8, vecs, (64, 64, 64), 1024,
                          APOD_UNIFORM, 1.0, c=c)


def mixed_geometries():
    """The mixed-grid ensemble: (grid, array side) pairs with 16 diverging waves."""
    out = []
    for dims, side in (((64, 64, 64), 16), ((96, 128, 64), 24), ((128, 128, 128), 32)):
        out.append(cfg2(dims=dims, n_side=side))
    return out


def sub_grid(g: Geometry, start, dims) -> Geometry:
    """The block of voxels [start, start+dims) of g, as a grid of its own."""
    o = np.asarray(g.grid_origin) + np.asarray(start) * np.asarray(g.grid_spacing)
    return g.replace(grid_origin=tuple(o), grid_dims=tuple(int(d) for d in dims))


def voxel_centre(g: Geometry, ix, iy, iz) -> np.ndarray:
    return (np.asarray(g.grid_origin, float)
            + np.asarray([ix, iy, iz], float) * np.asarray(g.grid_spacing, float))


# --------------------------------------------------------------------------
# scatterers
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Scatterers:
    pos: np.ndarray    # [L, 3]
    amp: np.ndarray    # [L]


def scatterers(g: Geometry, n_targets: int, n_speckle: int, seed_targets: int,
               seed_speckle: int, snap_targets: bool = False) -> Scatterers:
    """Point targets U(0.1, 1) inside the grid box shrunk by 4 voxels, plus
    N(0, 0.1^2)-amplitude speckle uniform over the grid box grown by 1 mm."""
    lo, hi = g.voxel_box()
    sp = np.asarray(g.grid_spacing, float)
    rt = np.random.default_rng(seed_targets)
    tlo, thi = lo + 4 * sp, hi - 4 * sp
    tpos = rt.uniform(tlo, thi, size=(n_targets, 3))
    if snap_targets:
        idx = np.rint((tpos - np.asarray(g.grid_origin)) / sp)
        tpos = np.asarray(g.grid_origin) + idx * sp
    tamp = rt.uniform(0.1, 1.0, size=n_targets)
    rs = np.random.default_rng(seed_speckle)
    spos = rs.uniform(lo - 1e-3, hi + 1e-3, size=(n_speckle, 3))
    samp = rs.normal(0.0, 0.1, size=n_speckle)
    return Scatterers(np.concatenate([tpos, spos]), np.concatenate([tamp, samp]))


def displaced(s: Scatterers, frame: int, seed_base: int, lam: float) -> Scatterers:
    """Random-walk displacement N(0, (lam/40)^2) per axis per frame."""
    pos = s.pos.copy()
    for f in range(1, frame + 1):
        r = np.random.default_rng(seed_base + f)
        pos = pos + r.normal(0.0, lam / 40.0, size=pos.shape)
    return Scatterers(pos, s.amp.copy())


# --------------------------------------------------------------------------
# channel-data simulator (ray model, Gaussian-modulated pulse)
# --------------------------------------------------------------------------

def pulse_sigma(fc: float = FC, bw: float = BANDWIDTH) -> float:
    """Gaussian envelope std whose -6 dB fractional bandwidth is bw."""
    return math.sqrt(2.0 * math.log(2.0)) / (math.pi * bw * fc)


def _tx_arrival_path(g: Geometry, s_pos):
    """Path length from the transmit time origin to each scatterer, [Q, L].

    This is the physics of the incident wave: a plane wave moving along u
    passes the origin at t = 0; a diverging wave leaves its virtual source v at
    t = 0.  tx_offset shifts the time origin by L/c."""
    import torch
    Q = g.Q
    out = []
    for q in range(Q):
        vec = torch.as_tensor(g.tx_vec[q], dtype=s_pos.dtype, device=s_pos.device)
        kind = int(g.tx_kind[q])
        if kind == TX_PLANE:
            d = s_pos @ vec
        elif kind == TX_DIVERGING:
            d = torch.linalg.norm(s_pos - vec, dim=-1)
        else:
            d = torch.zeros(s_pos.shape[0], dtype=s_pos.dtype, device=s_pos.device)
        out.append(d - float(g.tx_offset[q]))
    return torch.stack(out)


def simulate(g: Geometry, scat: Scatterers, c: Optional[float] = None,
             noise_std: float = 0.0, noise_seed: int = 0, normalize: bool = True,
             device: str = "cpu", half_taps: int = 12, dtype=None):
    """Channel data y[Q, M, K] (float32, torch) of point scatterers.

    Each scatterer returns a Gaussian-modulated pulse centred at its two-way
    travel time; samples are evaluated exactly at t0 + k/fs (no
    interpolation).  The result is normalised to max|y| = 1 before noise of
    std ``noise_std`` is added.  ``c`` defaults to the geometry's sound speed
    (the data may be made at another speed than the one used to image)."""
    import torch
    dt = torch.float64 if dtype is None else dtype
    c = g.c if c is None else float(c)
    Q, M, K = g.Q, g.M, g.K
    sig = pulse_sigma()
    spos = torch.as_tensor(scat.pos, dtype=dt, device=device)
    amp = torch.as_tensor(scat.amp, dtype=dt, device=device)
    epos = torch.as_tensor(g.elem_pos, dtype=dt, device=device)
    txp = _tx_arrival_path(g, spos)                                  # [Q, L]
    y = torch.zeros(Q, M * K, dtype=dt, device=device)
    offs = torch.arange(-half_taps, half_taps + 1, device=device, dtype=dt)
    T = offs.numel()
    budget = 4e7 if device == "cpu" else 1.5e8      # elements per temporary
    Lc = max(1, int(budget // (M * T)))
    for l0 in range(0, spos.shape[0], Lc):
        sp = spos[l0:l0 + Lc]
        a = amp[l0:l0 + Lc]
        rx = torch.cdist(epos, sp)                                   # [M, Lc]
        for q in range(Q):
            t = (txp[q, l0:l0 + Lc][None, :] + rx) / c               # [M, Lc] s
            ks = (t - g.t0) * g.fs
            k0 = torch.floor(ks)
            j = k0[..., None] + offs                                 # [M, Lc, T]
            tt = g.t0 + j / g.fs - t[..., None]
            v = a[None, :, None] * torch.exp(-0.5 * (tt / sig) ** 2) * torch.cos(2 * math.pi * FC * tt)
            valid = (j >= 0) & (j < K)
            flat = (torch.arange(M, device=device)[:, None, None] * K + j.clamp(0, K - 1).long())
            y[q].index_add_(0, flat[valid], v[valid])
    y = y.view(Q, M, K)
    if normalize:
        y = y / y.abs().max().clamp_min(1e-30)
    if noise_std > 0:
        gen = torch.Generator(device="cpu").manual_seed(noise_seed)
        y = y + noise_std * torch.randn(Q, M, K, generator=gen, dtype=dt).to(device)
    return y.to(torch.float32)


def cfg1_data(device="cpu"):
    g = cfg1()
    s = scatterers(g, 3, 0, seed_targets=1, seed_speckle=0, snap_targets=True)
    return g, s, simulate(g, s, noise_std=0.01, noise_seed=2, device=device)


def cfg2_data(device="cpu", geometry=None):
    g = cfg2() if geometry is None else geometry
    s = scatterers(g, 200, 10_000, seed_targets=3, seed_speckle=4)
    return g, s, simulate(g, s, device=device)


def cfg5_data(device="cpu"):
    g = cfg5()
    s = scatterers(g, 50, 2000, seed_targets=6, seed_speckle=60)
    return g, s, simulate(g, s, c=1500.0, device=device)


def motion_positions(s: Scatterers, frames: int, seed_base: int, lam: float):
    """Scatterer positions of frames 0 .. frames-1 of the random walk that
    ``displaced`` defines (frame f = displaced(s, f, seed_base, lam)),
    accumulated frame by frame."""
    pos = s.pos.copy()
    out = [pos.copy()]
    for f in range(1, frames):
        r = np.random.default_rng(seed_base + f)
        pos = pos + r.normal(0.0, lam / 40.0, size=pos.shape)
        out.append(pos.copy())
    return out


CFG4_SEED_BASE = 5


def cfg4_ensemble(frames: int = 256, device="cuda", which=None, g: Optional[Geometry] = None,
                  progress=None, dtype=None):
    """Doppler-style ensemble at the cfg2 geometry: the cfg2 scatterers (200
    targets, seed 3; 1e4 speckle, seed 4) moved by the per-frame random walk
    N(0, (lambda/40)^2) per axis (seed 5 + frame), each frame simulated and
    normalised like cfg2_data (frame 0 is the cfg2 frame).  Returns
    (g, y[F, Q, M, K] float32 on `device`, frame numbers), F = frames, or
    only the frames listed in ``which``.  ``progress(done, total)`` is called
    after every 32nd simulated frame; ``dtype`` is the simulator's working
    precision (FP64 by default; FP32 simulates a 256-frame ensemble several
    times faster, the arrival times then carrying ~1e-4 sample of rounding)."""
    import torch
    g = cfg2() if g is None else g
    s = scatterers(g, 200, 10_000, seed_targets=3, seed_speckle=4)
    lam = C_NOMINAL / FC
    pos = motion_positions(s, frames, CFG4_SEED_BASE, lam)
    ids = list(range(frames)) if which is None else [int(f) for f in which]
    y = torch.empty(len(ids), g.Q, g.M, g.K, dtype=torch.float32, device=device)
    for i, f in enumerate(ids):
        y[i] = simulate(g, Scatterers(pos[f], s.amp), device=device, dtype=dtype)
        if progress is not None and (i + 1) % 32 == 0:
            progress(i + 1, len(ids))
    return g, y, ids


def cfg5_focus_grid(g: Optional[Geometry] = None, oversample: int = 4) -> Geometry:
    """The cfg5 voxel grid sampled ``oversample`` times finer in depth over the
    same depth range (64 x 64 x 64 * oversample voxels): the envelope of an
    echo spans about one lambda/2 voxel in depth, so the autofocus criterion is
    evaluated on this grid to resolve it."""
    g = cfg5() if g is None else g
    sp = list(g.grid_spacing)
    sp[2] /= oversample
    nx, ny, nz = g.grid_dims
    return g.replace(grid_spacing=tuple(sp), grid_dims=(nx, ny, (nz - 1) * oversample + 1))


def random_channel_data(g: Geometry, batch: int, seed: int, device="cpu"):
    """y[B, Q, M, K] float32, i.i.d. N(0, 1): a stress input for parity."""
    import torch
    gen = torch.Generator(device="cpu").manual_seed(seed)
    return torch.randn(batch, g.Q, g.M, g.K, generator=gen).to(device)


def selective_tx_weights(g: Geometry, grid=None, overlap: float = 0.5, taper: float = 0.25):
    """Transmit weights w_tx[Q, N] float32 of a spatially selective sequence:
    the Q transmits are laid out on a lateral a x b grid (a b = Q; default the
    most square factorisation) and transmit (i, j) weighs only voxels whose
    lateral position falls inside its cell widened by `overlap` (fraction of a
    cell on each side), with a raised-cosine taper over the outer `taper`
    fraction of that box and exactly zero outside it.  An input pattern, not
    part of the beamformer: the forward treats it as any other w_tx."""
    Q = g.Q
    if grid is None:
        a = int(np.floor(np.sqrt(Q)))
        while Q % a:
            a -= 1
        grid = (Q // a, a)
    ga, gb = grid
    assert ga * gb == Q
    nx, ny, nz = g.grid_dims
    x = np.arange(nx) / max(nx - 1, 1)          # lateral position in [0, 1]
    y = np.arange(ny) / max(ny - 1, 1)

    def profile(u, cells, i):
        c0, c1 = i / cells, (i + 1) / cells
        half = 0.5 * (c1 - c0) * (1.0 + 2.0 * overlap)
        mid = 0.5 * (c0 + c1)
        d = np.abs(u - mid) / half                # 0 at the centre, 1 at the box edge
        w = np.where(d <= 1.0 - taper, 1.0,
                     np.where(d < 1.0, 0.5 * (1.0 + np.cos(np.pi * (d - (1.0 - taper)) / taper)), 0.0))
        return w

    w = np.empty((Q, nz, ny, nx), np.float32)
    for q in range(Q):
        i, j = q % ga, q // ga
        w[q] = (profile(y, gb, j)[:, None] * profile(x, ga, i)[None, :])[None, :, :]
    return w.reshape(Q, -1)


def doppler_ensemble(shape=(32, 24, 16), T: int = 64, seed: int = 0, n_clutter: int = 3,
                     clutter_amp: float = 100.0, blood_amp: float = 1.0, noise: float = 0.1,
                     rho: float = 0.9):
    """A synthetic beamformed Doppler ensemble x[T, N] float32 (N = prod(shape),
    n = ix + nx (iy + ny iz)): tissue clutter of rank n_clutter (smooth spatial
    patterns times slow temporal modulations, amplitude clutter_amp), blood
    inside a tube through the volume (AR(1) in time with coefficient rho,
    amplitude blood_amp) and white noise.  An input pattern only."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    N = nx * ny * nz
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    t = np.arange(T) / T
    x = np.zeros((T, N))
    for c in range(n_clutter):
        k = rng.uniform(0.5, 2.0, 3)
        ph = rng.uniform(0, 2 * np.pi, 3)
        spatial = (np.cos(2 * np.pi * k[0] * ix / nx + ph[0]) * np.cos(2 * np.pi * k[1] * iy / ny + ph[1])
                   * np.cos(2 * np.pi * k[2] * iz / nz + ph[2])).ravel()
        temporal = 1.0 + 0.3 * np.cos(2 * np.pi * (c + 0.5) * t + rng.uniform(0, 2 * np.pi))
        x += clutter_amp * (0.6 ** c) * temporal[:, None] * spatial[None, :]
    # blood: a tube along z at (nx/2, ny/3), radius ~ nx/6
    vessel = ((ix - nx / 2) ** 2 + (iy - ny / 3) ** 2 <= (nx / 6) ** 2).ravel()
    nb = int(vessel.sum())
    b = np.zeros((T, nb))
    b[0] = rng.normal(0, 1, nb)
    for i in range(1, T):
        b[i] = rho * b[i - 1] + np.sqrt(1 - rho ** 2) * rng.normal(0, 1, nb)
    x[:, vessel] += blood_amp * b
    x += noise * rng.normal(0, 1, (T, N))
    return x.astype(np.float32), vessel


def doppler_ensemble_device(shape=(128, 128, 128), T: int = 256, seed: int = 0, n_clutter: int = 3,
                            clutter_amp: float = 100.0, blood_amp: float = 1.0, noise: float = 0.1,
                            rho: float = 0.9, device="cuda"):
    """The recipe of doppler_ensemble generated with torch on a device (for
    ensembles too large for the host path); returns x[T, N] float32."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    nx, ny, nz = shape
    iz, iy, ix = torch.meshgrid(torch.arange(nz, device=device), torch.arange(ny, device=device),
                                torch.arange(nx, device=device), indexing="ij")
    t = torch.arange(T, device=device, dtype=torch.float32) / T
    x = torch.zeros(T, nx * ny * nz, device=device)
    for c in range(n_clutter):
        k = torch.rand(3, generator=g) * 1.5 + 0.5
        ph = torch.rand(4, generator=g) * 2 * np.pi
        spatial = (torch.cos(2 * np.pi * float(k[0]) * ix / nx + float(ph[0]))
                   * torch.cos(2 * np.pi * float(k[1]) * iy / ny + float(ph[1]))
                   * torch.cos(2 * np.pi * float(k[2]) * iz / nz + float(ph[2]))).reshape(-1)
        temporal = 1.0 + 0.3 * torch.cos(2 * np.pi * (c + 0.5) * t + float(ph[3]))
        x += clutter_amp * (0.6 ** c) * temporal[:, None] * spatial[None, :]
    vessel = ((ix - nx / 2) ** 2 + (iy - ny / 3) ** 2 <= (nx / 6) ** 2).reshape(-1)
    nb = int(vessel.sum())
    b = torch.randn(nb, generator=g).to(device)
    for i in range(T):
        if i:
            b = rho * b + float(np.sqrt(1 - rho ** 2)) * torch.randn(nb, generator=g).to(device)
        x[i, vessel] += blood_amp * b
    x += noise * torch.randn(T, nx * ny * nz, generator=g).to(device)
    return x.contiguous(), vessel

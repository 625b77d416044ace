"""Pins of ``oracle.nonzero_counts``: the numbers of (voxel, element) pairs and
(voxel, element, transmit) triples with a nonzero weight, the unit counts of
the algorithmic-work model that the benchmark's roofline divides by.

A pair has a nonzero Hann weight exactly when the voxel lies strictly inside
the element's receive cone: in front of the element (z > 0) and at a lateral
distance rho < z / (2F) (the receive-weight reading of the paragraph after
Eq. (1)).  Each test counts that set another way: by hand on a line of voxels,
by exact rational arithmetic on a lattice, by the cone's half-angle for a
tilted element, and on the full 128^3 x 1024 benchmark geometry by counting,
per voxel and element row, the element positions inside the chord the cone's
footprint cuts from that row.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _one_element(voxels_origin, spacing, dims, F=1.5, normal=None, Q=1):
    return synth.Geometry(
        elem_pos=np.zeros((1, 3)), elem_normal=None if normal is None else np.asarray([normal], float),
        tx_kind=np.full(Q, synth.TX_NONE, np.int32), tx_vec=np.zeros((Q, 3)), tx_offset=np.zeros(Q),
        grid_origin=tuple(voxels_origin), grid_spacing=tuple(spacing), grid_dims=tuple(dims),
        num_samples=16, c=1540.0, fs=30e6, apod=synth.APOD_HANN, f_number=F)


def test_line_of_voxels_through_the_cone():
    """One element at the origin facing +z, F = 1.5, voxels on the line z = 3 mm,
    x = -1.55 mm + i 0.1 mm (i < 32): the cone's radius there is 1 mm, so
    i = 6 .. 25 are inside: 20 pairs, and 20 Q triples for Q transmits."""
    g = _one_element((-1.55e-3, 0.0, 3e-3), (1e-4, 1e-4, 1e-4), (32, 1, 1), Q=5)
    pnz, tnz = oracle.nonzero_counts(g)
    assert (pnz, tnz) == (20, 100)
    # the same line behind the element sees nothing
    g_back = _one_element((-1.55e-3, 0.0, -3e-3), (1e-4, 1e-4, 1e-4), (32, 1, 1))
    assert oracle.nonzero_counts(g_back) == (0, 0)


def test_lattice_disc_exact():
    """A 41 x 37 x 3 block of voxels in front of one element: brute-force
    count of rho^2 < (z / 2F)^2 in exact rational arithmetic (coordinates in
    units of 0.1 mm, chosen off the cone's surface)."""
    F = Fraction(3, 2)
    ox, oy, oz = Fraction(-203, 10), Fraction(-181, 10), Fraction(53, 1)   # x 0.1 mm
    nx, ny, nz = 41, 37, 3
    zstep = Fraction(7, 1)
    count = 0
    for iz in range(nz):
        z = oz + iz * zstep
        a2 = (z / (2 * F)) ** 2
        for iy in range(ny):
            for ix in range(nx):
                x, yv = ox + ix, oy + iy
                count += (x * x + yv * yv) < a2
    g = _one_element((float(ox) * 1e-4, float(oy) * 1e-4, float(oz) * 1e-4), (1e-4, 1e-4, 7e-4),
                     (nx, ny, nz), F=1.5)
    assert 0 < count < nx * ny * nz
    assert oracle.nonzero_counts(g)[0] == count


def test_tilted_normal_half_angle():
    """An element tilted by 25 degrees about y: a voxel is inside exactly when
    the angle between (p - r) and the normal is below atan(1 / (2F))."""
    th = math.radians(25.0)
    n = np.array([math.sin(th), 0.0, math.cos(th)])
    F = 1.2
    g = _one_element((-2.0e-3, -1.5e-3, 2.0e-3), (1.3e-4, 1.1e-4, 1.7e-4), (31, 27, 9), F=F, normal=n)
    p = oracle.voxel_positions(g)
    cosang = (p @ n) / np.linalg.norm(p, axis=1)
    inside = np.arccos(np.clip(cosang, -1, 1)) < math.atan(1.0 / (2.0 * F))
    assert 0 < inside.sum() < g.N
    assert oracle.nonzero_counts(g)[0] == int(inside.sum())


def test_uniform_apodization_counts_every_pair():
    for g in (synth.cfg1(), synth.sub_grid(synth.cfg2(), (0, 0, 0), (4, 3, 2))):
        g = g.replace(apod=synth.APOD_UNIFORM)
        assert oracle.nonzero_counts(g) == (g.N * g.M, g.N * g.M * g.Q)


def _row_chord_count(g):
    """(voxel, element) pairs inside the receive cones of a flat +z-facing
    n x n array, counted per voxel and element row: the cone's footprint on
    the array plane is the disc of radius a = z / (2F) about the voxel's
    (x, y); element row j (at height y_j) meets it in the chord
    |x - x_p| < sqrt(a^2 - (y_j - y_p)^2), whose element count follows from the
    row's uniform spacing with a floor and a ceiling."""
    e = np.asarray(g.elem_pos)
    xs = np.unique(e[:, 0])
    ys = np.unique(e[:, 1])
    pitch = xs[1] - xs[0]
    nside = xs.size
    assert xs.size * ys.size == g.M and np.allclose(np.diff(xs), pitch) and np.allclose(e[:, 2], 0)
    nx, ny, nz = g.grid_dims
    o = np.asarray(g.grid_origin)
    sp = np.asarray(g.grid_spacing)
    px = o[0] + np.arange(nx) * sp[0]
    py = o[1] + np.arange(ny) * sp[1]
    total = 0
    for iz in range(nz):
        z = o[2] + iz * sp[2]
        a2 = (z / (2.0 * g.f_number)) ** 2
        dy2 = (ys[None, :] - py[:, None]) ** 2                      # [ny, rows]
        half = np.sqrt(np.maximum(a2 - dy2, 0.0))                    # chord half-length
        live = dy2 < a2
        # elements i with x_p - half < x0 + i pitch < x_p + half
        lo = (px[:, None, None] - half[None] - xs[0]) / pitch       # [nx, ny, rows]
        hi = (px[:, None, None] + half[None] - xs[0]) / pitch
        i_lo = np.maximum(np.floor(lo) + 1, 0)
        i_hi = np.minimum(np.ceil(hi) - 1, nside - 1)
        cnt = np.where(live[None], np.maximum(i_hi - i_lo + 1, 0), 0)
        total += int(cnt.sum())
    return total


def test_row_chords_match_oracle_on_a_block():
    g = synth.sub_grid(synth.cfg2(), (40, 50, 0), (24, 20, 6))
    assert oracle.nonzero_counts(g)[0] == _row_chord_count(g)


def test_benchmark_counts_golden():
    """tests/golden/nonzero_counts.json (written by make_counts.py with the
    oracle) against the row-chord count of the full cfg2 geometry, and the
    dense cfg1 / cfg5 cases (uniform apodization)."""
    with open(os.path.join(GOLDEN, "nonzero_counts.json")) as f:
        gold = json.load(f)
    g2 = synth.cfg2()
    assert gold["cfg2"]["pairs_nonzero"] == _row_chord_count(g2)
    assert gold["cfg2"]["triples_nonzero"] == 16 * gold["cfg2"]["pairs_nonzero"]
    for name, g in (("cfg1", synth.cfg1()), ("cfg5", synth.cfg5())):
        assert gold[name]["pairs_nonzero"] == g.N * g.M
        assert gold[name]["triples_nonzero"] == g.N * g.M * g.Q

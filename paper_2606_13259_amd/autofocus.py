"""Sound-speed autofocus with the differentiable delay-and-sum.

The focus criterion of a complex volume x~ beamformed at sound speed c from
analytic channel data (Re and Im lanes in one batch) is

    L(c) = sum_n |x~_n(c)|^4 / sum_n |x~_n(c)|^2,

the energy-weighted mean intensity.  It does not change when the image is
only magnified (both sums grow with the number of voxels an echo covers) and
it rises as the echoes focus, so its maximum marks the best-focused speed.
A plain energy sum_n |x~_n|^2 has no such maximum: on a grid fixed in metres
it grows with the assumed speed because every echo covers more voxels.
The criterion needs a grid that resolves each echo's envelope in depth (one
lambda/2 voxel is too coarse: sub-voxel shifts of the echoes then dominate).

The loop maximises L in two stages.  First it locates a zero of dL/dc:
dL/dc comes from the gradient kernel through ``DASFunction`` (nothing of the
volume or the delays is stored between forward and backward); the speed moves
uphill in growing steps until the slope changes sign, then the bracket is
halved on the sign of the slope until it is narrower than ``tol``.  L is
piecewise smooth (every interpolation tap that crosses a sample adds a kink)
and its broad maximum carries a ripple of about 0.1 % over 1-2 m/s, so the
slope can vanish at a ripple peak next to the highest one; the second stage
evaluates L on a ``grid`` m/s lattice within ``polish`` m/s of the bracket
and keeps the largest value.
"""
from __future__ import annotations

import torch

from . import das, metrics


def focus_criterion(plan: "das.Plan", lanes: torch.Tensor, c: torch.Tensor) -> torch.Tensor:
    """L(c) = sum |x~|^4 / sum |x~|^2 for analytic lanes [2, Q, M, K] (float32, on
    the plan's device); differentiable in c."""
    x = das.DASFunction.apply(lanes, c, plan)
    e2 = x[0].double() ** 2 + x[1].double() ** 2
    return (e2 * e2).sum() / e2.sum()


def value_and_slope(plan: "das.Plan", lanes: torch.Tensor, c: float):
    """(L(c), dL/dc) at one speed."""
    ct = torch.tensor(float(c), dtype=torch.float64, requires_grad=True)
    L = focus_criterion(plan, lanes, ct)
    L.backward()
    return float(L.detach()), float(ct.grad)


def autofocus(plan: "das.Plan", y: torch.Tensor, c0: float, bounds: tuple[float, float] = (1480.0, 1560.0),
              step: float = 4.0, tol: float = 0.25, max_evals: int = 60, grid: float = 0.5,
              polish: float = 4.0, lanes: torch.Tensor | None = None):
    """Maximise L(c) over ``bounds`` starting from c0 (m/s).

    y: real channel data [Q, M, K] (ignored when ``lanes`` is given).
    Returns (c, history) with history a list of (c, L, dL/dc) per slope
    evaluation; c is the best point of the final lattice (multiples of
    ``grid`` within ``polish`` of the slope bracket, inside ``bounds``)."""
    if plan.max_batch < 2:
        raise ValueError("autofocus needs a plan with max_batch >= 2 (Re and Im lanes)")
    if lanes is None:
        lanes = metrics.analytic_lanes(y).contiguous()
    lo_b, hi_b = float(bounds[0]), float(bounds[1])
    hist = []

    def ev(c):
        L, d = value_and_slope(plan, lanes, c)
        hist.append((c, L, d))
        return d

    def polished(lo, hi):
        import math
        a0 = max(lo_b, math.floor((lo - polish) / grid) * grid)
        cands = []
        v = a0
        while v <= min(hi_b, hi + polish) + 1e-9:
            if v >= lo_b - 1e-9:
                cands.append(v)
            v += grid
        best, best_L = cands[0], -float("inf")
        with torch.no_grad():
            for cv in cands:
                L = float(focus_criterion(plan, lanes, torch.tensor(cv, dtype=torch.float64)))
                if L > best_L:
                    best, best_L = cv, L
        return best

    c = min(max(float(c0), lo_b), hi_b)
    d = ev(c)
    direction = 1.0 if d > 0 else -1.0
    # walk uphill with doubling steps until the slope turns
    a, da = c, d
    b, db = a, da
    h = step
    while len(hist) < max_evals:
        b = min(max(a + direction * h, lo_b), hi_b)
        if b == a:                      # at a bound, slope still outward
            return polished(a, a), hist
        db = ev(b)
        if (db > 0) != (da > 0):
            break
        a, da = b, db
        h *= 2.0
    lo, hi = (a, b) if a < b else (b, a)
    d_lo = da if a < b else db
    # bisection on the sign of the slope (positive left of the maximum)
    while hi - lo > tol and len(hist) < max_evals:
        mid = 0.5 * (lo + hi)
        dm = ev(mid)
        if (dm > 0) == (d_lo > 0):
            lo, d_lo = mid, dm
        else:
            hi = mid
    return polished(lo, hi), hist

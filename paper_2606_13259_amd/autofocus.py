"""Sound-speed autofocus with the differentiable delay-and-sum.

The focus criterion is the envelope energy L(c) = sum_n |x~_n(c)|^2 of the
volume beamformed at sound speed c from analytic channel data (Re and Im lanes
in one batch).  It is largest when the delays match the medium.  The loop
ascends L with Adam; dL/dc comes from the gradient kernel through
``DASFunction`` (nothing of the volume or the delays is stored between
forward and backward).
"""
from __future__ import annotations

import torch

from . import das, metrics


def envelope_energy(plan: "das.Plan", lanes: torch.Tensor, c: torch.Tensor) -> torch.Tensor:
    """L(c) for analytic lanes [2, Q, M, K] (float32, on the plan's device)."""
    x = das.DASFunction.apply(lanes, c, plan)
    return (x.double() ** 2).sum()


def autofocus(plan: "das.Plan", y: torch.Tensor, c0: float, steps: int = 80, lr: float = 3.0,
              decay: float = 0.95, lanes: torch.Tensor | None = None,
              bounds: tuple[float, float] | None = None):
    """Maximise the envelope energy over c, starting from c0 (m/s), with Adam
    and an exponentially decaying step (lr * decay^t, in m/s); with
    ``bounds`` = (c_min, c_max) every step is projected onto that interval.

    y: real channel data [Q, M, K] (ignored when ``lanes`` is given).
    Returns (c, history) with history a list of (c, L) per step."""
    if plan.max_batch < 2:
        raise ValueError("autofocus needs a plan with max_batch >= 2 (Re and Im lanes)")
    if lanes is None:
        lanes = metrics.analytic_lanes(y).contiguous()
    c = torch.tensor(float(c0), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([c], lr=lr)
    sched = torch.optim.lr_scheduler.ExponentialLR(opt, gamma=decay)
    hist = []
    L0 = None
    for _ in range(steps):
        opt.zero_grad()
        L = envelope_energy(plan, lanes, c)
        if L0 is None:
            L0 = float(L.detach())
        (-L / L0).backward()           # ascend; normalised so lr is in m/s
        hist.append((float(c.detach()), float(L.detach())))
        opt.step()
        if bounds is not None:
            with torch.no_grad():
                c.clamp_(float(bounds[0]), float(bounds[1]))
        sched.step()
    return float(c.detach()), hist

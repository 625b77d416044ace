"""The Doppler-style ensemble at full size: 256 frames of the 128^3 x 1024 x 16
geometry whose scatterers move by a seeded sub-wavelength random walk per
frame, in the forms and launches the benchmark times.  Frames 0, 1, 128 and 255
(first and last 64-item batch-tile groups, neighbouring items and the middle
of the batch) are simulated; the other items hold seeded random data, so a
mix-up between items shows.  Checked against the FP64 oracle on sampled voxels
computed one by one, on the raw FP32 data (storage + kernel error) and on the
values the workspace holds (kernel error alone)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import check_close, lowp_bars, round_like_storage, sample_voxels, say

pytestmark = pytest.mark.gpu

FRAMES = (0, 1, 128, 255)
B = 256
KERNEL_REL, KERNEL_ABS = 5e-4, 1e-3  # f16 interpolation weights (relative rounding <= 2^-11)


def _das():
    from paper_2606_13259_amd import das
    return das


_CACHE = {}


def _ensemble(gpu):
    if "y" not in _CACHE:
        g, ys, ids = synth.cfg4_ensemble(B, device=gpu, which=FRAMES)
        gen = torch.Generator(device=gpu).manual_seed(77)
        y = 0.05 * torch.randn(B, g.Q, g.M, g.K, device=gpu, generator=gen)
        for i, f in enumerate(ids):
            y[f] = ys[i]
        idx = sample_voxels(g, 384, seed=4)
        ysel = y[list(FRAMES)].cpu().numpy()
        _CACHE.update(g=g, y=y, idx=idx, ysel=ysel, xo=oracle.forward(ysel, g, voxels=idx))
    return _CACHE


def _check_frames(x, c, storage, what):
    g, idx, ysel, xo = c["g"], c["idx"], c["ysel"], c["xo"]
    xr = oracle.forward(round_like_storage(ysel, storage), g, voxels=idx)
    xs = x[list(FRAMES)][:, torch.from_numpy(idx).to(x.device)].cpu().numpy()
    assert np.all(np.isfinite(xs))
    for i, f in enumerate(FRAMES):
        check_close(xs[i], xo[i], *lowp_bars(storage), f"{what} frame {f}, sampled voxels")
        check_close(xs[i], xr[i], KERNEL_REL, KERNEL_ABS, f"  {what} frame {f}, rounded data")


def test_motion_frames_are_distinct(gpu):
    """The random walk moves the scatterers: consecutive frames differ, but by
    far less than the echo itself (sub-wavelength motion)."""
    c = _ensemble(gpu)
    y = c["y"]
    d01 = float((y[1] - y[0]).norm() / y[0].norm())
    d0_255 = float((y[255] - y[0]).norm() / y[0].norm())
    say(f"  |y1 - y0|/|y0| = {d01:.3e}, |y255 - y0|/|y0| = {d0_255:.3e}")
    assert 1e-4 < d01 < 0.5
    assert d0_255 > d01


@pytest.mark.parametrize("storage,form", [("f16", "auto"), ("f16", "slab"), ("fp8", "auto"),
                                          ("fp8", "slab")])
def test_ensemble_256_frames_mfma(gpu, storage, form):
    das = _das()
    c = _ensemble(gpu)
    plan = das.Plan(c["g"], max_batch=B, storage=storage)
    plan.set_mfma_form(form)
    assert plan.algo(B) == "mfma"
    say(f"cfg4 ensemble: {B} motion frames, {storage} MFMA, {form} form")
    x = plan.forward(c["y"])
    _check_frames(x, c, storage, f"{storage} mfma {form}")
    plan.close()


def test_ensemble_in_mixed_persistent_launch(gpu):
    """The 256-frame ensemble and the mixed grids (64^3 / 256 el, 96x128x64 /
    576 el, 128^3 / 1024 el, 16 frames each) in ONE persistent launch: the
    ensemble equals its own launch bit for bit and the oracle on the frames."""
    das = _das()
    c = _ensemble(gpu)
    plan = das.Plan(c["g"], max_batch=B, storage="f16")
    plans, wss, batches = [plan], [plan.prepare(c["y"])], [B]
    for i, gm in enumerate(synth.mixed_geometries()):
        pm = das.Plan(gm, max_batch=16, storage="f16")
        wss.append(pm.prepare(synth.random_channel_data(gm, 16, seed=90 + i, device=gpu)))
        plans.append(pm)
        batches.append(16)
    xs = [torch.full((b, p.N), float("nan"), device=gpu) for p, b in zip(plans, batches)]
    say("cfg4 ensemble + mixed grids in one persistent launch")
    das.das_forward_batched([p.handle for p in plans], wss, batches, xs)
    for p, ws, x, b in zip(plans, wss, xs, batches):
        assert torch.equal(x, p.forward_ws(ws, b)), "persistent launch differs from a separate launch"
    _check_frames(xs[0], c, "f16", "persistent")
    for p in plans:
        p.close()

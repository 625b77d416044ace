"""FP8 (E4M3) workspace storage against the FP64 oracle (MI355X).

Two bars per case: against the oracle on the raw FP32 data (storage plus
kernel error, the storage-limited FP8 bar) and against the oracle on the values
the workspace holds (oracle.storage: E4M3 rounding with one power-of-two scale
per item), which leaves the kernel error alone: FP32 level for the windowed
form (the decode is exact and the arithmetic FP32), the f16-weight level for
the MFMA form (samples decode exactly to f16 operands, weights are rounded to
f16)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import (ABS_F32, REL_L2_F32, cfg2_channel_data, check_close, lowp_bars,
                            round_like_storage, sample_voxels, say)

pytestmark = pytest.mark.gpu

KERNEL = {"tiled": (REL_L2_F32, ABS_F32), "mfma": (5e-4, 1e-3)}


def _das():
    from paper_2606_13259_amd import das
    return das


def _geometry():
    g = synth.cfg2(dims=(13, 9, 7), n_side=8).replace(num_samples=1500)
    return g.replace(tx_kind=np.array([synth.TX_DIVERGING, synth.TX_PLANE, synth.TX_NONE], np.int32),
                     tx_vec=np.array([[0.6e-3, -0.4e-3, -8e-3], synth.plane_wave(6, -4), [0, 0, 0]]),
                     tx_offset=np.array([7e-3, 0.0, -5e-3]))


def _items(g, B, seed):
    """B items at amplitudes spread over 60 orders of magnitude: each item is
    scaled by its own power of two, so every one keeps the same accuracy."""
    y = synth.random_channel_data(g, B, seed=seed)
    amps = torch.tensor([1.0, 1e-3, 5e4, 1e-30, 3e30, 0.25, 7.0, 1e-12][:B] + [1.0] * max(0, B - 8))
    return (y * amps[:B, None, None, None]).contiguous()


def _check(x, y_np, g, algo, idx, what):
    xo = oracle.forward(y_np, g)
    xr = oracle.forward(round_like_storage(y_np, "fp8"), g)
    for i, b in enumerate(idx):
        check_close(x[b], xo[i], *lowp_bars("fp8"), f"{what} b={b}")
        check_close(x[b], xr[i], *KERNEL[algo], f"  oracle on fp8-rounded data b={b}")


@pytest.mark.parametrize("algo,B", [("tiled", 1), ("tiled", 5), ("mfma", 16), ("mfma", 17),
                                    ("mfma", 40)])
def test_fp8_items_at_any_amplitude(gpu, algo, B):
    das = _das()
    g = _geometry()
    y = _items(g, B, seed=60 + B)
    say(f"fp8 {algo} B={B}")
    plan = das.Plan(g, max_batch=B, storage="fp8")
    assert plan.algo(B) == algo
    x = plan.forward(y.to(gpu)).cpu().numpy()
    idx = list(range(min(B, 5))) + ([B - 1] if B > 5 else [])
    _check(x, y.numpy()[idx], g, algo, idx, f"fp8 {algo}")


@pytest.mark.parametrize("B", [5, 20])
def test_fp8_prepare_in_slices(gpu, B):
    """A workspace prepared in two slices (each finding its own items' scales)
    equals one prepared at once: the same scale table (the last 4 B bytes:
    each item's largest magnitude) and the same output bit for bit.  (Padding
    items and alignment bytes are never written, so raw bytes are not
    compared.)"""
    das = _das()
    g = synth.cfg2(dims=(8, 8, 4), n_side=8).replace(num_samples=1200)
    y = _items(g, B, seed=9).to(gpu)
    plan = das.Plan(g, max_batch=B, storage="fp8")
    ws1 = plan.prepare(y)
    ws2 = plan.workspace(B)
    das.das_prepare(plan.handle, y[:3].contiguous(), 0, 3, B, ws2)
    das.das_prepare(plan.handle, y[3:].contiguous(), 3, B - 3, B, ws2)
    torch.cuda.synchronize()
    t1, t2 = ws1[-4 * B:].view(torch.float32), ws2[-4 * B:].view(torch.float32)
    assert torch.equal(t1, t2)
    assert torch.equal(t1.cpu(), y.abs().amax(dim=(1, 2, 3)).cpu())
    assert torch.equal(plan.forward_ws(ws1, B), plan.forward_ws(ws2, B))


@pytest.mark.parametrize("B", [4, 16])
def test_fp8_special_items(gpu, B):
    """An all-zero item gives zeros; an item with NaN samples (every sample
    of its first transmit, so that every voxel reads some) is stored unscaled
    and yields NaN without touching the other items."""
    das = _das()
    g = _geometry()
    y = synth.random_channel_data(g, B, seed=70)
    y[0] = 0.0
    y[1, 0] = float("nan")
    plan = das.Plan(g, max_batch=B, storage="fp8")
    x = plan.forward(y.to(gpu)).cpu().numpy()
    assert np.all(x[0] == 0.0)
    assert np.any(np.isnan(x[1]))
    assert np.all(np.isfinite(x[2:]))
    idx = [2, B - 1]
    _check(x, y.numpy()[idx], g, plan.algo(B), idx, "fp8 next to special items")


def test_fp8_persistent_batched(gpu):
    """One persistent launch per algorithm over FP8 plans equals separate
    launches bit for bit."""
    das = _das()
    for geoms, batches in (([_geometry(), synth.cfg1()], [40, 16]),
                           ([_geometry(), synth.cfg1()], [3, 2])):
        plans, wss, xs = [], [], []
        for g, B in zip(geoms, batches):
            p = das.Plan(g, max_batch=B, storage="fp8")
            wss.append(p.prepare(_items(g, B, seed=80 + B).to(gpu)))
            plans.append(p)
            xs.append(torch.full((B, p.N), float("nan"), device=gpu))
        say(f"fp8 batched {[p.algo(B) for p, B in zip(plans, batches)]}")
        das.das_forward_batched([p.handle for p in plans], wss, batches, xs)
        for p, ws, x, B in zip(plans, wss, xs, batches):
            assert torch.equal(x, p.forward_ws(ws, B))


@pytest.mark.parametrize("algo,B", [("tiled", 1), ("mfma", 16)])
def test_fp8_cfg2_full_volume_sampled(gpu, algo, B):
    """The full 128^3 x 1024 x 16 geometry in the benchmark's launch
    configuration (AUTO), on sampled voxels computed one by one."""
    das = _das()
    g, y = cfg2_channel_data()
    yb = torch.cat([y[None], synth.random_channel_data(g, B - 1, seed=41, device=y.device)]).contiguous()
    plan = das.Plan(g, max_batch=B, storage="fp8")
    assert plan.algo(B) == algo
    say(f"fp8 cfg2 full volume {algo} B={B}")
    x = plan.forward(yb)
    items = [0, B - 1] if B > 1 else [0]
    x = x[items].cpu().numpy()
    idx = sample_voxels(g, 256, seed=18)
    ynp = yb[items].cpu().numpy()
    xo = oracle.forward(ynp, g, voxels=idx)
    xr = oracle.forward(round_like_storage(ynp, "fp8"), g, voxels=idx)
    for i, b in enumerate(items):
        check_close(x[i][idx], xo[i], *lowp_bars("fp8"), f"item {b}, sampled voxels")
        check_close(x[i][idx], xr[i], *KERNEL[algo], "  oracle on fp8-rounded data")


def test_mfma_launches_overlapping_on_two_streams(gpu):
    """Persistent MFMA forwards of one plan enqueued on two streams at once
    take different counter sets: both equal a lone launch bit for bit."""
    das = _das()
    g = _geometry()
    B = 40
    plan = das.Plan(g, max_batch=B, storage="fp8")
    ws = plan.prepare(_items(g, B, seed=90).to(gpu))
    ref = plan.forward_ws(ws, B)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for r in range(3):
        for s in (s1, s2):
            with torch.cuda.stream(s):
                x = torch.full_like(ref, float("nan"))
                das.das_forward(plan.handle, ws, B, x)  # on the current stream s
                outs.append(x)
    torch.cuda.synchronize()
    for x in outs:
        assert torch.equal(x, ref)

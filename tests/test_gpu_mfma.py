"""Matrix-core (MFMA) locality form against the FP64 oracle (MI355X).

Two bars per case: against the oracle on the raw FP32 data (storage plus
kernel error: 1e-3 for FP16, the storage-limited 4e-3 for BF16), and against
the oracle on the values
the workspace holds (kernel error alone: f16 weights carry a relative
rounding of at most 2^-11, bf16 weights are split into two bf16 parts and
carry at most about 2^-16)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import (cfg2_channel_data, check_close, lowp_bars, round_like_storage,
                            sample_voxels, say)

pytestmark = pytest.mark.gpu

# kernel error alone (oracle on the rounded data)
KERNEL_REL = {"f16": 5e-4, "bf16": 5e-5}
KERNEL_ABS = {"f16": 1e-3, "bf16": 1e-4}


def _das():
    from paper_2606_13259_amd import das
    return das


def _check_both(x, y_np, g, storage, what, w_tx=None):
    xo = oracle.forward(y_np, g, w_tx=w_tx)
    xr = oracle.forward(round_like_storage(y_np, storage), g, w_tx=w_tx)
    for b in range(x.shape[0]):
        check_close(x[b], xo[b], *lowp_bars(storage), f"{what} b={b}")
        check_close(x[b], xr[b], KERNEL_REL[storage], KERNEL_ABS[storage], f"  rounded data b={b}")


def _ragged_geometry():
    g = synth.cfg2(dims=(13, 9, 7), n_side=8).replace(num_samples=1500)
    return g.replace(tx_kind=np.array([synth.TX_DIVERGING, synth.TX_PLANE, synth.TX_NONE], np.int32),
                     tx_vec=np.array([[0.6e-3, -0.4e-3, -8e-3], synth.plane_wave(6, -4), [0, 0, 0]]),
                     tx_offset=np.array([7e-3, 0.0, -5e-3]))


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("B", [1, 16, 17, 40])
def test_mfma_ragged_batches(gpu, storage, B):
    """Grid not a multiple of the 4x4 voxel group, three transmit kinds (padded
    to a transmit group of 4), batch sizes on both sides of the 16-column MFMA
    tile (1, 2 and 4 tiles per wavefront, padded columns)."""
    das = _das()
    g = _ragged_geometry()
    y = synth.random_channel_data(g, B, seed=20 + B)
    say(f"mfma ragged 13x9x7, Q=3, B={B}, {storage}")
    plan = das.Plan(g, max_batch=B, storage=storage, algo="mfma")
    assert plan.algo(B) == "mfma"
    x = plan.forward(y.to(gpu)).cpu().numpy()
    items = range(B) if B <= 4 else (0, B // 2, B - 1)
    idx = list(items)
    _check_both(x[idx], y.numpy()[idx], g, storage, f"B={B}")


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_mfma_cfg2_subblocks(gpu, storage):
    """Simulated cfg2 data (with a second, random item) on a block near the
    array and a deep block."""
    das = _das()
    g, y = cfg2_channel_data()
    yb = torch.stack([y, synth.random_channel_data(g, 1, seed=31, device=y.device)[0]]).contiguous()
    ynp = yb.cpu().numpy()
    for start, dims in (((40, 52, 0), (20, 12, 10)), ((70, 30, 100), (17, 16, 9))):
        sub = synth.sub_grid(g, start, dims)
        say(f"mfma cfg2 block start={start} dims={dims} {storage}")
        plan = das.Plan(sub, max_batch=2, storage=storage, algo="mfma")
        x = plan.forward(yb).cpu().numpy()
        _check_both(x, ynp, sub, storage, f"cfg2 block {dims}")


def test_mfma_cfg1_plane_wave_uniform(gpu):
    """One plane wave, uniform apodization (no culling), 64 elements."""
    das = _das()
    g, _, y = synth.cfg1_data()
    yb = torch.stack([y, 0.5 * y.flip(-1)]).contiguous()
    plan = das.Plan(g, max_batch=2, storage="f16", algo="mfma")
    x = plan.forward(yb.to(gpu)).cpu().numpy()
    _check_both(x, yb.numpy(), g, "f16", "cfg1")


def test_mfma_transmit_weights(gpu):
    das = _das()
    g = synth.cfg2(dims=(9, 8, 6), n_side=6).replace(num_samples=1800)
    B = 16
    y = synth.random_channel_data(g, B, seed=5)
    w = np.random.default_rng(6).uniform(0.0, 1.0, size=(g.Q, g.N)).astype(np.float32)
    plan = das.Plan(g, max_batch=B, storage="f16", algo="mfma")
    plan.set_tx_weights(torch.from_numpy(w).to(gpu))
    x = plan.forward(y.to(gpu)).cpu().numpy()
    _check_both(x[[0, 9, 15]], y.numpy()[[0, 9, 15]], g, "f16", "w_tx", w_tx=w)


def test_mfma_partial_prepare_and_auto_choice(gpu):
    """AUTO picks MFMA for 16-bit storage from 16 items; a workspace prepared
    in two slices equals one prepared at once; f32 storage refuses MFMA."""
    das = _das()
    g = synth.cfg2(dims=(8, 8, 4), n_side=8).replace(num_samples=1200)
    B = 20
    y = synth.random_channel_data(g, B, seed=9).to(gpu)
    plan = das.Plan(g, max_batch=B, storage="f16")
    assert plan.algo(B) == "mfma" and plan.algo(15) == "tiled"
    ws1 = plan.prepare(y)
    ws2 = plan.workspace(B)
    das.das_prepare(plan.handle, y[:7].contiguous(), 0, 7, B, ws2)
    das.das_prepare(plan.handle, y[7:].contiguous(), 7, B - 7, B, ws2)
    x1 = plan.forward_ws(ws1, B)
    x2 = plan.forward_ws(ws2, B)
    assert torch.equal(x1, x2)
    f32 = das.Plan(g, max_batch=B, storage="f32")
    assert f32.algo(B) == "tiled"
    with pytest.raises(das.DasError) as e:
        f32.set_algo("mfma")
    assert e.value.status == das.DAS_ERR_UNSUPPORTED
    with pytest.raises(das.DasError) as e:
        das.Plan(g, max_batch=B, storage="f32", algo="mfma")
    assert e.value.status == das.DAS_ERR_UNSUPPORTED


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_mfma_cfg2_full_volume_sampled(gpu, storage):
    """The full 128^3 x 1024 x 16 geometry at 16 items in the benchmark's
    launch configuration (AUTO), on sampled voxels computed one by one."""
    das = _das()
    g, y = cfg2_channel_data()
    B = 16
    yb = torch.cat([y[None], synth.random_channel_data(g, B - 1, seed=40, device=y.device)]).contiguous()
    plan = das.Plan(g, max_batch=B, storage=storage)
    assert plan.algo(B) == "mfma"
    say(f"mfma cfg2 full volume, B={B}, {storage}")
    x = plan.forward(yb)
    items = [0, 7, 15]
    x = x[items].cpu().numpy()
    assert np.all(np.isfinite(x))
    idx = sample_voxels(g, 256, seed=17)
    ynp = yb[items].cpu().numpy()
    xo = oracle.forward(ynp, g, voxels=idx)
    xr = oracle.forward(round_like_storage(ynp, storage), g, voxels=idx)
    for i, b in enumerate(items):
        check_close(x[i][idx], xo[i], *lowp_bars(storage), f"item {b}, sampled voxels")
        check_close(x[i][idx], xr[i], KERNEL_REL[storage], KERNEL_ABS[storage], "  rounded data")


def test_mfma_persistent_batched_launch(gpu):
    """One persistent MFMA launch over plans with different grids, arrays,
    transmit counts and batch sizes (different column tiles per wavefront)
    equals separate launches bit for bit, and the oracle within the bars."""
    das = _das()
    geoms = [_ragged_geometry(),
             synth.sub_grid(synth.cfg5(), (20, 24, 10), (9, 8, 12)),
             synth.cfg1()]
    batches = [40, 17, 16]
    plans, wss, xs, ys = [], [], [], []
    for g, B in zip(geoms, batches):
        y = synth.random_channel_data(g, B, seed=50 + B)
        p = das.Plan(g, max_batch=B, storage="f16")
        assert p.algo(B) == "mfma"
        ws = p.prepare(y.to(gpu))
        plans.append(p)
        wss.append(ws)
        xs.append(torch.full((B, p.N), float("nan"), device=gpu))
        ys.append(y)
    das.das_forward_batched([p.handle for p in plans], wss, batches, xs)
    for p, ws, x, y, g, B in zip(plans, wss, xs, ys, geoms, batches):
        xsep = p.forward_ws(ws, B)
        assert torch.equal(x, xsep), "batched launch differs from a separate launch"
        idx = [0, B - 1]
        _check_both(x[idx].cpu().numpy(), y.numpy()[idx], g, "f16", f"batched {g.grid_dims}")
    # plans of different algorithms cannot share one launch
    g = geoms[2]
    p_t = das.Plan(g, max_batch=2, storage="f16")
    ws_t = p_t.prepare(synth.random_channel_data(g, 2, seed=3).to(gpu))
    with pytest.raises(das.DasError) as e:
        das.das_forward_batched([plans[2].handle, p_t.handle], [wss[2], ws_t], [16, 2],
                                [xs[2], torch.empty(2, p_t.N, device=gpu)])
    assert e.value.status == das.DAS_ERR_UNSUPPORTED

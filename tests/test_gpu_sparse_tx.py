"""Sparse transmit lists (the paper's sparse observation lists, Sec. 5) on the
MI355X: with transmit weights, a voxel tile (windowed kernel) or column (MFMA
form) skips the transmits whose weight is zero everywhere in it.  The skipped
terms are exact zeros, so the output is the oracle's with the same weights."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import ABS_F32, REL_L2_F32, check_close, lowp_bars, say

pytestmark = pytest.mark.gpu


def _das():
    from paper_2606_13259_amd import das
    return das


def _block(dims=(20, 12, 10), start=(40, 52, 30)):
    return synth.sub_grid(synth.cfg2(), start, dims)


@pytest.mark.parametrize("storage,algo,B", [("f32", "tiled", 1), ("f32", "tiled", 3),
                                            ("f16", "mfma", 16), ("fp8", "mfma", 40)])
def test_selective_transmits(gpu, storage, algo, B):
    """A spatially selective sequence (each of the 16 transmits weighs one
    lateral cell of a 4 x 4 layout, widened and tapered, zero elsewhere)."""
    das = _das()
    g = _block()
    w = synth.selective_tx_weights(g)
    say(f"selective w_tx: {(w > 0).mean():.2f} of (q, n) nonzero; {storage} {algo} B={B}")
    y = synth.random_channel_data(g, B, seed=100 + B)
    plan = das.Plan(g, max_batch=B, storage=storage, algo=algo)
    plan.set_tx_weights(torch.from_numpy(w).to(gpu))
    x = plan.forward(y.to(gpu)).cpu().numpy()
    idx = [0, B - 1] if B > 1 else [0]
    xo = oracle.forward(y.numpy()[idx], g, w_tx=w)
    bars = (REL_L2_F32, ABS_F32) if storage == "f32" else lowp_bars(storage)
    for i, b in enumerate(idx):
        check_close(x[b], xo[i], *bars, f"b={b}")


@pytest.mark.parametrize("algo,storage,B", [("tiled", "f32", 2), ("mfma", "f16", 16)])
def test_region_without_transmits_is_zero(gpu, algo, storage, B):
    """Weights zero for every transmit on one half of the volume: that half is
    exactly zero, the other half matches the oracle."""
    das = _das()
    g = _block((16, 12, 8))
    w = np.ones((g.Q, g.N), np.float32)
    ix = np.arange(g.N) % g.grid_dims[0]
    w[:, ix < 8] = 0.0
    y = synth.random_channel_data(g, B, seed=7)
    plan = das.Plan(g, max_batch=B, storage=storage, algo=algo)
    plan.set_tx_weights(torch.from_numpy(w).to(gpu))
    x = plan.forward(y.to(gpu)).cpu().numpy()
    assert np.all(x[:, ix < 8] == 0.0)
    xo = oracle.forward(y.numpy()[:1], g, w_tx=w)
    bars = (REL_L2_F32, ABS_F32) if storage == "f32" else lowp_bars(storage)
    check_close(x[0], xo[0], *bars, "half-lit volume")


def test_many_transmits_keep_the_dense_path(gpu):
    """More than 64 transmits: the windowed kernel keeps its dense transmit
    loop (the per-tile list holds 64); results still match the oracle."""
    das = _das()
    g0 = _block((9, 8, 6))
    Q = 72
    rng = np.random.default_rng(5)
    vecs = np.stack([rng.uniform(-4e-3, 4e-3, Q), rng.uniform(-4e-3, 4e-3, Q), np.full(Q, -10e-3)], 1)
    g = g0.replace(tx_kind=np.full(Q, synth.TX_DIVERGING, np.int32), tx_vec=vecs,
                   tx_offset=np.zeros(Q), num_samples=1200)
    w = rng.uniform(0, 1, (Q, g.N)).astype(np.float32) * (rng.uniform(0, 1, (Q, 1)) > 0.5)
    y = synth.random_channel_data(g, 1, seed=8)
    plan = das.Plan(g, max_batch=1, storage="f32", algo="tiled")
    plan.set_tx_weights(torch.from_numpy(w).to(gpu))
    x = plan.forward(y.to(gpu)).cpu().numpy()
    xo = oracle.forward(y.numpy(), g, w_tx=w)
    check_close(x[0], xo[0], REL_L2_F32, ABS_F32, "Q = 72")


def test_sparse_lists_in_persistent_launch(gpu):
    """Windowed plans with selective weights in one persistent launch equal
    separate launches bit for bit."""
    das = _das()
    geoms = [_block((20, 12, 10)), _block((16, 16, 8), start=(10, 10, 60))]
    plans, wss, xs, bs = [], [], [], [2, 3]
    for g, B in zip(geoms, bs):
        p = das.Plan(g, max_batch=B, storage="f32", algo="tiled")
        p.set_tx_weights(torch.from_numpy(synth.selective_tx_weights(g)).to(gpu))
        wss.append(p.prepare(synth.random_channel_data(g, B, seed=B).to(gpu)))
        xs.append(torch.full((B, p.N), float("nan"), device=gpu))
        plans.append(p)
    das.das_forward_batched([p.handle for p in plans], wss, bs, xs)
    for p, ws, x, B in zip(plans, wss, xs, bs):
        assert torch.equal(x, p.forward_ws(ws, B))

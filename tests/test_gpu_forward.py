"""Forward-pass parity of the HIP path against the FP64 oracle (MI355X)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import (ABS_F32, REL_L2_F32, cfg2_channel_data, check_close, lowp_bars, rel_l2,
                            round_like_storage, sample_voxels, say)

pytestmark = pytest.mark.gpu


def _das():
    from paper_2606_13259_amd import das
    return das


@pytest.mark.parametrize("algo", ["plain", "tiled"])
def test_cfg1_f32(gpu, algo):
    das = _das()
    g, _, y = synth.cfg1_data()
    say(f"cfg1 16^3 x 64 x 1, algo={algo}")
    plan = das.Plan(g, max_batch=1, storage="f32", algo=algo)
    assert plan.algo(1) == algo
    x = plan.forward(y[None].to(gpu)).cpu().numpy()[0]
    xo = oracle.forward(y.numpy()[None], g)[0]
    check_close(x, xo, REL_L2_F32, ABS_F32, f"cfg1 {algo}")


@pytest.mark.parametrize("algo", ["plain", "tiled"])
@pytest.mark.parametrize("B", [2, 3, 5])
def test_batches_and_ragged_grid(gpu, algo, B):
    """Random data, several batch items, a grid that is not a multiple of any
    tile, Hann apodization and two transmit kinds."""
    das = _das()
    g = synth.cfg2(dims=(13, 9, 7), n_side=8).replace(num_samples=1500)
    g = g.replace(tx_kind=np.array([synth.TX_DIVERGING, synth.TX_PLANE, synth.TX_NONE], np.int32),
                  tx_vec=np.array([[0.6e-3, -0.4e-3, -8e-3], synth.plane_wave(6, -4), [0, 0, 0]]),
                  tx_offset=np.array([7e-3, 0.0, -5e-3]))
    y = synth.random_channel_data(g, B, seed=10 + B)
    say(f"ragged 13x9x7, B={B}, algo={algo}")
    plan = das.Plan(g, max_batch=B, storage="f32", algo=algo)
    x = plan.forward(y.to(gpu)).cpu().numpy()
    xo = oracle.forward(y.numpy(), g)
    for b in range(B):
        check_close(x[b], xo[b], REL_L2_F32, ABS_F32, f"b={b}")


@pytest.fixture(scope="module")
def cfg2_blocks():
    """Two cfg2 sub-blocks (near the array, deep) with their oracle volumes."""
    g, y = cfg2_channel_data()
    yc = y.cpu().numpy()[None]
    out = []
    for start, dims in (((40, 52, 0), (20, 12, 10)), ((70, 30, 100), (17, 16, 9))):
        sub = synth.sub_grid(g, start, dims)
        say(f"oracle cfg2 block start={start} dims={dims}")
        out.append((sub, oracle.forward(yc, sub)[0]))
    return g, y, out


@pytest.mark.parametrize("storage,algo", [("f32", "plain"), ("f32", "tiled"), ("f16", "tiled"),
                                          ("bf16", "tiled"), ("fp8", "tiled")])
def test_cfg2_subblocks(gpu, cfg2_blocks, storage, algo):
    das = _das()
    g, y, blocks = cfg2_blocks
    for sub, xo in blocks:
        plan = das.Plan(sub, max_batch=1, storage=storage, algo=algo)
        x = plan.forward(y[None].to(gpu)).cpu().numpy()[0]
        if storage == "f32":
            check_close(x, xo, REL_L2_F32, ABS_F32, f"cfg2 block {sub.grid_dims} {storage} {algo}")
        else:
            check_close(x, xo, *lowp_bars(storage), f"cfg2 block {sub.grid_dims} {storage} {algo}")
            # kernel error alone: oracle on the values the workspace holds
            xr = oracle.forward(round_like_storage(y.cpu().numpy()[None], storage), sub)[0]
            check_close(x, xr, REL_L2_F32, ABS_F32, f"  vs oracle on {storage}-rounded data")


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16", "fp8"])
def test_one_item_staging_short_odd_record(gpu, storage):
    """One-item windows are staged four samples per lane; with K = 41 (odd,
    shorter than a window) and t0 = 13.5 us, 12 % of the taps fall before the
    record and 11 % after it, so staging takes its per-sample path at both
    ends and its four-sample loads start at every alignment."""
    das = _das()
    g = synth.cfg2(dims=(11, 9, 13), n_side=8).replace(num_samples=41, t0=13.5e-6)
    y = synth.random_channel_data(g, 1, seed=41)
    plan = das.Plan(g, max_batch=1, storage=storage, algo="tiled")
    x = plan.forward(y.to(gpu)).cpu().numpy()[0]
    xo = oracle.forward(y.numpy(), g)[0]
    if storage == "f32":
        check_close(x, xo, REL_L2_F32, ABS_F32, "K=41 f32")
    else:
        check_close(x, xo, *lowp_bars(storage), f"K=41 {storage}")
        xr = oracle.forward(round_like_storage(y.numpy(), storage), g)[0]
        check_close(x, xr, REL_L2_F32, ABS_F32, f"  vs oracle on {storage}-rounded data")


def test_cfg2_full_volume_sampled(gpu):
    """The full 128^3 x 1024 x 16 volume in the benchmark's launch
    configuration, checked on sampled voxels computed one by one."""
    das = _das()
    g, y = cfg2_channel_data()
    plan = das.Plan(g, max_batch=1, storage="f32")
    say(f"cfg2 full volume, algo={plan.algo(1)}, tile={das.das_tile_shape(plan.tile())}")
    assert plan.algo(1) == "tiled"
    x = plan.forward(y[None].contiguous()).cpu().numpy()[0]
    assert np.all(np.isfinite(x))
    idx = sample_voxels(g, 768, seed=7)
    xo = oracle.forward(y.cpu().numpy()[None], g, voxels=idx)[0]
    check_close(x[idx], xo, REL_L2_F32, ABS_F32, "cfg2 full, sampled voxels")


def test_delay_formation_error(gpu):
    """The kernels' fractional sample index vs the FP64 oracle's, cfg2."""
    das = _das()
    g, y = cfg2_channel_data()
    plan = das.Plan(g, max_batch=1, storage="f32")
    worst = 0.0
    p_all = None
    for q in (0, 5, 15):
        for n0 in (0, 1_000_000, g.N - 4096):
            f = plan.debug_delays(q, 0, g.M, n0, n0 + 4096).cpu().numpy()
            p = oracle.voxel_positions(g, np.arange(n0, n0 + 4096))
            fo = oracle.fractional_index(oracle.transmit_path(g, p)[q][None, :],
                                         oracle.receive_path(g, p), g.c, g.fs, g.t0)
            worst = max(worst, float(np.max(np.abs(f - fo))))
    say(f"  max |f_kernel - f_oracle| = {worst:.3e} samples")
    assert worst <= 1e-3


def test_edge_cases(gpu):
    das = _das()
    cases = []
    # one voxel, one element, one transmit, K = 2, taps straddling both ends
    base = synth.Geometry(elem_pos=np.zeros((1, 3)), elem_normal=None,
                          tx_kind=np.array([synth.TX_NONE], np.int32), tx_vec=np.zeros((1, 3)),
                          tx_offset=np.zeros(1), grid_origin=(0.0, 0.0, 3e-3),
                          grid_spacing=(1e-4, 1e-4, 1e-4), grid_dims=(1, 1, 1), num_samples=2,
                          c=1500.0, fs=30e6)
    for t0 in (3e-3 / 1500 - 0.5 / 30e6, 3e-3 / 1500 + 0.25 / 30e6, 3e-3 / 1500 - 1.25 / 30e6,
               3e-3 / 1500 + 5 / 30e6, 3e-3 / 1500 - 3 / 30e6):
        cases.append(("K=2 t0", base.replace(t0=t0)))
    # thin grids, single element, tilted normals with Hann
    g = synth.cfg2(dims=(1, 37, 3), n_side=1).replace(num_samples=3000)
    cases.append(("1x37x3, M=1", g))
    g = synth.cfg2(dims=(33, 1, 1), n_side=4).replace(num_samples=3000, f_number=0.7)
    rng = np.random.default_rng(3)
    nrm = np.tile([0.0, 0.0, 1.0], (16, 1)) + rng.normal(0, 0.15, (16, 3))
    cases.append(("33x1x1 tilted normals", g.replace(elem_normal=nrm)))
    for name, g in cases:
        y = synth.random_channel_data(g, 1, seed=4)
        xo = oracle.forward(y.numpy(), g)[0]
        for algo in ("plain", "tiled"):
            plan = das.Plan(g, max_batch=1, storage="f32", algo=algo)
            x = plan.forward(y.to(gpu)).cpu().numpy()[0]
            if np.max(np.abs(xo)) == 0:
                assert np.max(np.abs(x)) == 0, name
            else:
                check_close(x, xo, REL_L2_F32, ABS_F32, f"{name} {algo}")


def test_transmit_weights(gpu):
    das = _das()
    g = synth.cfg2(dims=(9, 8, 6), n_side=6).replace(num_samples=1800)
    y = synth.random_channel_data(g, 2, seed=5)
    w = np.random.default_rng(6).uniform(0.0, 1.0, size=(g.Q, g.N)).astype(np.float32)
    xo = oracle.forward(y.numpy(), g, w_tx=w)
    for algo in ("plain", "tiled"):
        plan = das.Plan(g, max_batch=2, storage="f32", algo=algo)
        wt = torch.from_numpy(w).to(gpu)
        plan.set_tx_weights(wt)
        x = plan.forward(y.to(gpu)).cpu().numpy()
        for b in range(2):
            check_close(x[b], xo[b], REL_L2_F32, ABS_F32, f"w_tx {algo} b={b}")


def test_autotune_and_every_tile_shape(gpu):
    """Every candidate tile shape meets the FP32 bar; autotuning picks one."""
    das = _das()
    g = synth.cfg2(dims=(19, 17, 9))
    y = synth.random_channel_data(g, 1, seed=8)
    xo = oracle.forward(y.numpy(), g)[0]
    y = y.to(gpu)
    plan = das.Plan(g, max_batch=1, storage="f32", algo="tiled")
    t = plan.autotune(1)
    say(f"  autotuned tile {das.das_tile_shape(t)}")
    ran = []
    for ti in range(das.das_num_tile_shapes()):
        try:
            plan.set_tile(ti)
        except das.DasError as e:
            # shapes whose sample windows exceed one lane per sample are refused
            assert e.status == das.DAS_ERR_UNSUPPORTED
            say(f"  tile {das.das_tile_shape(ti)}: unsupported for this geometry")
            continue
        assert plan.algo(1) == "tiled"
        check_close(plan.forward(y).cpu().numpy()[0], xo, REL_L2_F32, ABS_F32,
                    f"tile {das.das_tile_shape(ti)}")
        ran.append(ti)
    assert 0 in ran and t in ran


def test_workspace_layout_is_stable(gpu):
    """Regression: refusing a tile shape must not change the workspace layout
    that das_forward expects (a half-size f16 workspace was once read as an
    f32 plain-layout one)."""
    das = _das()
    g = synth.cfg2(dims=(16, 16, 8), n_side=16)
    B = 6
    y = synth.random_channel_data(g, B, seed=12)
    xo = oracle.forward(y.numpy(), g)
    plan = das.Plan(g, max_batch=B, storage="f16")
    ws = plan.prepare(y.to(gpu))
    assert ws.numel() == B * g.Q * g.M * g.K * 2
    refused = 0
    for ti in range(das.das_num_tile_shapes()):
        before = plan.tile()
        try:
            plan.set_tile(ti)
        except das.DasError as e:
            assert e.status == das.DAS_ERR_UNSUPPORTED
            assert plan.tile() == before
            refused += 1
        assert plan.algo(B) == "tiled"
        x = plan.forward_ws(ws, B).cpu().numpy()
        for b in (0, B - 1):
            check_close(x[b], xo[b], *lowp_bars("f16"), f"tile {das.das_tile_shape(plan.tile())}")
    assert refused > 0


def test_persistent_batched_launch(gpu):
    """One persistent launch over plans with different grids, arrays,
    transmit counts and batch sizes equals separate launches and the oracle."""
    das = _das()
    geoms = [synth.cfg2(dims=(13, 10, 7), n_side=8).replace(num_samples=1600),
             synth.sub_grid(synth.cfg5(), (20, 24, 10), (9, 8, 12)),
             synth.cfg1()]
    batches = [2, 3, 1]
    plans, wss, xs, ys = [], [], [], []
    for g, B in zip(geoms, batches):
        y = synth.random_channel_data(g, B, seed=20 + B)
        p = das.Plan(g, max_batch=B, storage="f32")
        ws = p.prepare(y.to(gpu))
        plans.append(p)
        wss.append(ws)
        xs.append(torch.full((B, p.N), float("nan"), device=gpu))
        ys.append(y)
    das.das_forward_batched([p.handle for p in plans], wss, batches, xs)
    for p, ws, x, y, g, B in zip(plans, wss, xs, ys, geoms, batches):
        xsep = p.forward_ws(ws, B)
        assert torch.equal(x, xsep), "batched launch differs from a separate launch"
        xo = oracle.forward(y.numpy(), g)
        for b in range(B):
            check_close(x[b].cpu().numpy(), xo[b], REL_L2_F32, ABS_F32, f"batched {g.grid_dims} b={b}")


@pytest.mark.parametrize("algo,storage,B", [("plain", "f32", 3), ("tiled", "f32", 3),
                                             ("tiled", "f16", 5), ("mfma", "f16", 17),
                                             ("tiled", "fp8", 3), ("mfma", "fp8", 17)])
def test_unusual_sizes(gpu, algo, storage, B):
    """Element count not a multiple of the 64-lane culling blocks or the 512-entry
    element passes (M = 1100), more transmits than one compile-time group
    (Q = 20, three kinds), an odd K, an odd grid."""
    das = _das()
    rng = np.random.default_rng(77)
    base = synth.cfg2(dims=(7, 5, 9), n_side=8)
    pos = np.concatenate([synth.matrix_array(32, 0.3e-3), rng.uniform(-5e-3, 5e-3, (76, 3)) * [1, 1, 0]])
    kinds = np.array([synth.TX_DIVERGING, synth.TX_PLANE, synth.TX_NONE, synth.TX_PLANE] * 5, np.int32)
    vecs = []
    for i, k in enumerate(kinds):
        if k == synth.TX_DIVERGING:
            vecs.append([rng.uniform(-3e-3, 3e-3), rng.uniform(-3e-3, 3e-3), -10e-3])
        elif k == synth.TX_PLANE:
            vecs.append(synth.plane_wave(rng.uniform(-8, 8), rng.uniform(-8, 8)))
        else:
            vecs.append([0.0, 0.0, 0.0])
    g = base.replace(elem_pos=pos, elem_normal=None, tx_kind=kinds, tx_vec=np.array(vecs),
                     tx_offset=rng.uniform(0, 5e-3, 20) * (kinds == synth.TX_DIVERGING),
                     num_samples=1000, t0=2e-6)
    y = synth.random_channel_data(g, B, seed=78)
    say(f"unusual sizes M={g.M} Q={g.Q} K={g.K} grid={g.grid_dims} {algo} {storage} B={B}")
    plan = das.Plan(g, max_batch=B, storage=storage, algo=algo)
    x = plan.forward(y.to(gpu)).cpu().numpy()
    items = [0, B - 1]
    ynp = y.numpy()[items]
    xo = oracle.forward(ynp, g)
    for i, b in enumerate(items):
        if storage == "f32":
            check_close(x[b], xo[i], REL_L2_F32, ABS_F32, f"b={b}")
        else:
            check_close(x[b], xo[i], *lowp_bars(storage), f"b={b}")

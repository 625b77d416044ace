"""The launch forms of the MFMA algorithm (das_plan_set_mfma_form: 4 x 4 x 4
columns, 8 x 8 x 1 slabs, the persistent kernel) against the FP64 oracle, with
the bars of tests/test_gpu_mfma.py: storage plus kernel error against the
oracle on the raw data, kernel error alone against the oracle on the values
the workspace holds.  Cases cover 1, 2 and 4 MFMA tiles per wavefront, grids
that are not multiples of the wavefront boxes, transmit weights, the full
128^3 x 1024 x 16 geometry, and the autotuner's choice."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import (cfg2_channel_data, check_close, lowp_bars, round_like_storage,
                            sample_voxels, say)

pytestmark = pytest.mark.gpu

KERNEL_REL = {"f16": 5e-4, "bf16": 5e-5, "fp8": 5e-4}
KERNEL_ABS = {"f16": 1e-3, "bf16": 1e-4, "fp8": 1e-3}
# FP8 matrix operands: each interpolation weight (scaled by 2^7) is carried
# as two E4M3 parts, a relative error of at most 2^-8 (2^-9 on average with
# round to nearest) instead of the f16 weights' 2^-11; on incoherent (random)
# data the output error is of that relative size: bars 4e-3 / 8e-3.
KERNEL_FP8W = (4e-3, 8e-3)
FORMS = ["column", "slab", "persistent"]


def _das():
    from paper_2606_13259_amd import das
    return das


def _check_both(x, y_np, g, storage, what, w_tx=None, kernel=None):
    xo = oracle.forward(y_np, g, w_tx=w_tx)
    xr = oracle.forward(round_like_storage(y_np, storage), g, w_tx=w_tx)
    kb = kernel or (KERNEL_REL[storage], KERNEL_ABS[storage])
    for b in range(x.shape[0]):
        check_close(x[b], xo[b], *lowp_bars(storage), f"{what} b={b}")
        check_close(x[b], xr[b], *kb, f"  rounded data b={b}")


def _ragged_geometry():
    g = synth.cfg2(dims=(19, 13, 7), n_side=8).replace(num_samples=1500)
    return g.replace(tx_kind=np.array([synth.TX_DIVERGING, synth.TX_PLANE, synth.TX_NONE], np.int32),
                     tx_vec=np.array([[0.6e-3, -0.4e-3, -8e-3], synth.plane_wave(6, -4), [0, 0, 0]]),
                     tx_offset=np.array([7e-3, 0.0, -5e-3]))


def _plan(g, B, storage, form):
    das = _das()
    p = das.Plan(g, max_batch=B, storage=storage, algo="mfma")
    p.set_mfma_form(form)
    assert p.mfma_form() == form and p.algo(B) == "mfma"
    return p


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("storage", ["f16", "bf16", "fp8"])
@pytest.mark.parametrize("B", [16, 40])
def test_forms_ragged(gpu, form, storage, B):
    g = _ragged_geometry()
    y = synth.random_channel_data(g, B, seed=130 + B)
    say(f"mfma {form} ragged {g.grid_dims}, Q=3, B={B}, {storage}")
    x = _plan(g, B, storage, form).forward(y.to(gpu)).cpu().numpy()
    idx = [0, B // 2, B - 1]
    _check_both(x[idx], y.numpy()[idx], g, storage, f"{form} B={B}")


@pytest.mark.parametrize("form", ["slab", "persistent"])
def test_forms_transmit_weights(gpu, form):
    g = synth.cfg2(dims=(17, 10, 6), n_side=6).replace(num_samples=1800)
    B = 32
    y = synth.random_channel_data(g, B, seed=15)
    w = np.random.default_rng(16).uniform(0.0, 1.0, size=(g.Q, g.N)).astype(np.float32)
    w[:, ::3] = 0.0
    p = _plan(g, B, "f16", form)
    p.set_tx_weights(torch.from_numpy(w).to(gpu))
    x = p.forward(y.to(gpu)).cpu().numpy()
    _check_both(x[[0, 31]], y.numpy()[[0, 31]], g, "f16", f"{form} w_tx", w_tx=w)


@pytest.mark.parametrize("storage", ["f16", "fp8"])
def test_slab_cfg2_full_volume_sampled(gpu, storage):
    g, y = cfg2_channel_data()
    B = 64
    yb = torch.cat([y[None], synth.random_channel_data(g, B - 1, seed=42, device=y.device)]).contiguous()
    say(f"mfma slab cfg2 full volume, B={B}, {storage}")
    x = _plan(g, B, storage, "slab").forward(yb)
    items = [0, 31, 63]
    x = x[items].cpu().numpy()
    assert np.all(np.isfinite(x))
    idx = sample_voxels(g, 256, seed=19)
    ynp = yb[items].cpu().numpy()
    xo = oracle.forward(ynp, g, voxels=idx)
    xr = oracle.forward(round_like_storage(ynp, storage), g, voxels=idx)
    for i, b in enumerate(items):
        check_close(x[i][idx], xo[i], *lowp_bars(storage), f"item {b}, sampled voxels")
        check_close(x[i][idx], xr[i], KERNEL_REL[storage], KERNEL_ABS[storage], "  rounded data")


def test_forms_agree(gpu):
    """All forms read one workspace; they agree to the f16 weight rounding."""
    das = _das()
    g = synth.sub_grid(synth.cfg2(), (50, 40, 60), (24, 20, 9))
    B = 32
    y = synth.random_channel_data(g, B, seed=8).to(gpu)
    p = das.Plan(g, max_batch=B, storage="f16", algo="mfma")
    ws = p.prepare(y)
    out = {}
    for form in FORMS:
        p.set_mfma_form(form)
        out[form] = p.forward_ws(ws, B)
    for form in ("slab", "persistent"):
        r = float((out[form] - out["column"]).norm() / out["column"].norm())
        say(f"  {form} vs column rel-L2 {r:.2e}")
        assert r <= 5e-4


def test_autotune_picks_an_mfma_form(gpu):
    das = _das()
    g = synth.sub_grid(synth.cfg2(), (40, 40, 40), (32, 32, 8))
    p = das.Plan(g, max_batch=32, storage="f16")
    assert p.algo(32) == "mfma" and p.mfma_form() == "auto"
    p.autotune(32)
    assert p.mfma_form() in FORMS
    with pytest.raises(das.DasError) as e:
        das._check(das.lib().das_plan_set_mfma_form(p.handle, 7), "das_plan_set_mfma_form")
    assert e.value.status == das.DAS_ERR_INVALID_ARG


@pytest.mark.parametrize("form", ["column_fp8", "slab_fp8"])
@pytest.mark.parametrize("B", [16, 40])
def test_fp8_operand_forms(gpu, form, B):
    """FP8 storage contracted on the FP8 matrix instructions (E4M3 weights)."""
    g = _ragged_geometry()
    y = synth.random_channel_data(g, B, seed=140 + B)
    say(f"mfma {form} ragged {g.grid_dims}, B={B}")
    x = _plan(g, B, "fp8", form).forward(y.to(gpu)).cpu().numpy()
    idx = [0, B // 2, B - 1]
    _check_both(x[idx], y.numpy()[idx], g, "fp8", f"{form} B={B}", kernel=KERNEL_FP8W)


def test_fp8_operand_cfg2_full_volume_sampled(gpu):
    g, y = cfg2_channel_data()
    B = 64
    yb = torch.cat([y[None], synth.random_channel_data(g, B - 1, seed=43, device=y.device)]).contiguous()
    say(f"mfma slab_fp8 cfg2 full volume, B={B}")
    x = _plan(g, B, "fp8", "slab_fp8").forward(yb)
    items = [0, 63]
    x = x[items].cpu().numpy()
    idx = sample_voxels(g, 256, seed=20)
    ynp = yb[items].cpu().numpy()
    xo = oracle.forward(ynp, g, voxels=idx)
    xr = oracle.forward(round_like_storage(ynp, "fp8"), g, voxels=idx)
    for i, b in enumerate(items):
        check_close(x[i][idx], xo[i], *lowp_bars("fp8"), f"item {b}, sampled voxels")
        check_close(x[i][idx], xr[i], *KERNEL_FP8W, "  rounded data")


def test_fp8_operand_forms_need_fp8_storage(gpu):
    das = _das()
    p = das.Plan(_ragged_geometry(), max_batch=16, storage="f16", algo="mfma")
    with pytest.raises(das.DasError) as e:
        p.set_mfma_form("slab_fp8")
    assert e.value.status == das.DAS_ERR_UNSUPPORTED

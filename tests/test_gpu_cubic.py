"""Four-point Lagrange (cubic) interpolation in the windowed kernel against the
FP64 oracle's cubic forward (reading R15), at the FP32 bars: rel-L2 <= 1e-5
and max |x - x_o| / max |x_o| <= 1e-5."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import ABS_F32, REL_L2_F32, cfg2_channel_data, check_close, sample_voxels, say

pytestmark = pytest.mark.gpu


def _das():
    from paper_2606_13259_amd import das
    return das


def _ragged_geometry():
    g = synth.cfg2(dims=(13, 9, 7), n_side=8).replace(num_samples=1500)
    return g.replace(tx_kind=np.array([synth.TX_DIVERGING, synth.TX_PLANE, synth.TX_NONE], np.int32),
                     tx_vec=np.array([[0.6e-3, -0.4e-3, -8e-3], synth.plane_wave(6, -4), [0, 0, 0]]),
                     tx_offset=np.array([7e-3, 0.0, -5e-3]))


@pytest.mark.parametrize("B", [1, 3])
def test_cubic_ragged_geometry(gpu, B):
    das = _das()
    g = _ragged_geometry()
    y = synth.random_channel_data(g, B, seed=60 + B)
    say(f"cubic ragged 13x9x7, Q=3, B={B}")
    plan = das.Plan(g, max_batch=B, storage="f32")
    plan.set_interp("cubic")
    x = plan.forward(y.to(gpu)).cpu().numpy()
    xo = oracle.forward(y.numpy(), g, interp="cubic")
    for b in range(B):
        check_close(x[b], xo[b], REL_L2_F32, ABS_F32, f"cubic B={B} b={b}")
    # linear interpolation of the same data differs (the option takes effect)
    plan.set_interp("linear")
    xl = plan.forward(y.to(gpu)).cpu().numpy()
    assert np.linalg.norm(xl - x) > 1e-3 * np.linalg.norm(x)


def test_cubic_record_ends(gpu):
    """cfg1: 5.5 % of the taps fall past the end of the 256-sample record, so
    the cubic taps k-1 and k+2 read the zero padding at both ends."""
    das = _das()
    g, _, y = synth.cfg1_data()
    yb = torch.stack([y, y.flip(-1)]).contiguous()
    plan = das.Plan(g, max_batch=2, storage="f32")
    plan.set_interp("cubic")
    x = plan.forward(yb.to(gpu)).cpu().numpy()
    xo = oracle.forward(yb.numpy(), g, interp="cubic")
    for b in range(2):
        check_close(x[b], xo[b], REL_L2_F32, ABS_F32, f"cubic cfg1 b={b}")


def test_cubic_cfg2_full_volume_sampled(gpu):
    """The full 128^3 x 1024 x 16 geometry with simulated data, sampled voxels."""
    das = _das()
    g, y = cfg2_channel_data()
    plan = das.Plan(g, max_batch=1, storage="f32")
    plan.set_interp("cubic")
    say("cubic cfg2 full volume, B=1")
    x = plan.forward(y[None].contiguous())[0]
    idx = sample_voxels(g, 512, seed=23)
    xo = oracle.forward(y.cpu().numpy()[None], g, voxels=idx, interp="cubic")[0]
    check_close(x[torch.from_numpy(idx).to(gpu)].cpu().numpy(), xo, REL_L2_F32, ABS_F32,
                "cubic cfg2 sampled voxels")


def test_cubic_refusals(gpu):
    das = _das()
    g = synth.cfg1()
    p16 = das.Plan(g, max_batch=1, storage="f16")
    with pytest.raises(das.DasError) as e:
        p16.set_interp("cubic")
    assert e.value.status == das.DAS_ERR_UNSUPPORTED
    p = das.Plan(g, max_batch=1, storage="f32")
    p.set_interp("cubic")
    with pytest.raises(das.DasError) as e:
        p.adjoint(torch.zeros(1, p.N, device=gpu))
    assert e.value.status == das.DAS_ERR_UNSUPPORTED
    with pytest.raises(das.DasError) as e:
        p.set_algo("plain")
    assert e.value.status == das.DAS_ERR_UNSUPPORTED
    p.set_interp("linear")
    p.set_algo("plain")
    with pytest.raises(das.DasError) as e:
        p.set_interp("cubic")
    assert e.value.status == das.DAS_ERR_UNSUPPORTED

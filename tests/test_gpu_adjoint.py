"""Adjoint, sound-speed gradient and autograd parity on the MI355X."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import ABS_F32, REL_L2_F32, check_close, rel_l2, say

pytestmark = pytest.mark.gpu


def _das():
    from paper_2606_13259_amd import das
    return das


def _small():
    g = synth.cfg2(dims=(14, 10, 9), n_side=8).replace(num_samples=1400)
    return g.replace(tx_kind=np.array([synth.TX_DIVERGING, synth.TX_PLANE], np.int32),
                     tx_vec=np.array([[0.5e-3, 0.2e-3, -9e-3], synth.plane_wave(-5, 3)]),
                     tx_offset=np.array([8e-3, 0.0]))


@pytest.mark.parametrize("geom", ["cfg1", "small"])
def test_adjoint_vs_oracle(gpu, geom):
    das = _das()
    g = synth.cfg1() if geom == "cfg1" else _small()
    B = 2
    gx = np.random.default_rng(1).normal(size=(B, g.N)).astype(np.float32)
    gyo = oracle.adjoint(gx, g)
    plan = das.Plan(g, max_batch=B, storage="f32")
    gy = plan.adjoint(torch.from_numpy(gx).to(gpu)).cpu().numpy()
    for b in range(B):
        check_close(gy[b].ravel(), gyo[b].ravel(), REL_L2_F32, ABS_F32, f"adjoint {geom} b={b}")


def test_dot_product_fp32(gpu):
    das = _das()
    g = _small()
    rng = np.random.default_rng(2)
    y = torch.from_numpy(rng.normal(size=(1, g.Q, g.M, g.K)).astype(np.float32)).to(gpu)
    x = torch.from_numpy(rng.normal(size=(1, g.N)).astype(np.float32)).to(gpu)
    for algo in ("plain", "tiled"):
        plan = das.Plan(g, max_batch=1, storage="f32", algo=algo)
        lhs = float((plan.forward(y).double() * x.double()).sum())
        rhs = float((y.double() * plan.adjoint(x).double()).sum())
        say(f"  <Ay,x>={lhs:.9e} <y,A^T x>={rhs:.9e} ({algo})")
        assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("geom", ["cfg5_block", "small"])
def test_grad_sound_speed_vs_oracle(gpu, geom):
    das = _das()
    if geom == "cfg5_block":
        g = synth.sub_grid(synth.cfg5(), (24, 24, 20), (12, 10, 8))
    else:
        g = _small()
    rng = np.random.default_rng(3)
    y = rng.normal(size=(2, g.Q, g.M, g.K)).astype(np.float32)
    gx = rng.normal(size=(2, g.N)).astype(np.float32)
    ref = oracle.grad_sound_speed(y, gx, g)
    plan = das.Plan(g, max_batch=2, storage="f32")
    got = float(plan.grad_sound_speed(torch.from_numpy(y).to(gpu), torch.from_numpy(gx).to(gpu)))
    say(f"  dL/dc gpu={got:.7e} oracle={ref:.7e}")
    assert abs(got - ref) <= 1e-4 * abs(ref)


def test_autograd_function(gpu):
    das = _das()
    g = synth.sub_grid(synth.cfg5(), (28, 28, 24), (8, 8, 8))
    rng = np.random.default_rng(4)
    y = torch.from_numpy(rng.normal(size=(1, g.Q, g.M, g.K)).astype(np.float32)).to(gpu)
    y.requires_grad_(True)
    c = torch.tensor(1530.0, dtype=torch.float64, requires_grad=True)
    plan = das.Plan(g, max_batch=1, storage="f32")
    x = das.DASFunction.apply(y, c, plan)
    w = torch.from_numpy(rng.normal(size=x.shape).astype(np.float32)).to(gpu)
    loss = (x * w).sum()
    loss.backward()
    plan.set_sound_speed(1530.0)
    gy_ref = plan.adjoint(w)
    assert rel_l2(y.grad.cpu().numpy().ravel(), gy_ref.cpu().numpy().ravel()) < 1e-6
    gc_ref = oracle.grad_sound_speed(y.detach().cpu().numpy(), w.cpu().numpy(), g, c=1530.0)
    say(f"  autograd dL/dc={float(c.grad):.7e} oracle={gc_ref:.7e}")
    assert abs(float(c.grad) - gc_ref) <= 1e-4 * abs(gc_ref)


def test_adjoint_cfg5_full_size_sampled_channels(gpu):
    """The adjoint at the full differentiable-case size (64^3 voxels, 16x16
    array, 8 plane waves, Re and Im lanes) in the launch the benchmark times,
    checked on sampled channels: the oracle adjoint of a geometry that holds
    only the sampled elements gives gy[b, q, m, :] for those elements and every
    transmit (the rows of A^T for element m depend on that element alone)."""
    das = _das()
    g = synth.cfg5()
    B = 2
    rng = np.random.default_rng(11)
    gx = rng.normal(size=(B, g.N)).astype(np.float32)
    plan = das.Plan(g, max_batch=B, storage="f32")
    say(f"adjoint cfg5 full size {g.grid_dims} x {g.M} el x {g.Q} tx, B={B}")
    gy = plan.adjoint(torch.from_numpy(gx).to(gpu)).cpu().numpy()
    assert gy.shape == (B, g.Q, g.M, g.K)
    sel = np.sort(rng.choice(g.M, size=6, replace=False))
    sel = np.unique(np.concatenate([sel, [0, g.M - 1, g.M // 2 + 8]]))
    sub = g.replace(elem_pos=np.asarray(g.elem_pos)[sel],
                    elem_normal=None if g.elem_normal is None else np.asarray(g.elem_normal)[sel])
    gyo = oracle.adjoint(gx, sub)
    for b in range(B):
        check_close(gy[b][:, sel].ravel(), gyo[b].ravel(), REL_L2_F32, ABS_F32,
                    f"adjoint cfg5 b={b}, elements {sel.tolist()}")

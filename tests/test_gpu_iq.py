"""Complex baseband (IQ) beamforming and its transpose on the MI355X against
the FP64 oracle (oracle.iq.forward_iq, oracle.iq.adjoint_iq).  The phase
rotation is formed from FP64 per-tile phase terms plus an FP32 tile-relative
part (a few 1e-7 revolutions) and the hardware sine and cosine of the
revolution count (in the windowed forward, of its transmit and element parts
separately, whose phasors are multiplied); the bar is the FP32 one (rel-L2
and elementwise 1e-5 against the FP64 oracle)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle.iq import adjoint_iq, demodulate, forward_iq
from paper_2606_13259_amd import metrics
from tests.gpu_util import ABS_F32, REL_L2_F32, cfg2_channel_data, check_close, say

pytestmark = pytest.mark.gpu


def _das():
    from paper_2606_13259_amd import das
    return das


def _geometry():
    g = synth.cfg2(dims=(13, 9, 7), n_side=8).replace(num_samples=1500, t0=1.5e-6)
    return g.replace(tx_kind=np.array([synth.TX_DIVERGING, synth.TX_PLANE, synth.TX_NONE], np.int32),
                     tx_vec=np.array([[0.6e-3, -0.4e-3, -8e-3], synth.plane_wave(6, -4), [0, 0, 0]]),
                     tx_offset=np.array([7e-3, 0.0, -5e-3]))


def _run(g, y_iq, fc, gpu, w_tx=None):
    """y_iq complex [C, Q, M, K] -> GPU x complex [C, N] (I/Q interleaved items)."""
    das = _das()
    C = y_iq.shape[0]
    lanes = np.empty((2 * C,) + y_iq.shape[1:], np.float32)
    lanes[0::2] = y_iq.real
    lanes[1::2] = y_iq.imag
    plan = das.Plan(g, max_batch=2 * C, storage="f32", algo="tiled")
    plan.set_iq(fc)
    if w_tx is not None:
        plan.set_tx_weights(torch.from_numpy(w_tx).to(gpu))
    x = plan.forward(torch.from_numpy(lanes).to(gpu)).cpu().numpy().astype(np.float64)
    return x[0::2] + 1j * x[1::2]


def _check(x, xo, what):
    for c in range(x.shape[0]):
        check_close(np.concatenate([x[c].real, x[c].imag]), np.concatenate([xo[c].real, xo[c].imag]),
                    REL_L2_F32, ABS_F32, f"{what} item {c}")


@pytest.mark.parametrize("C,fc", [(1, 7.5e6), (3, 7.5e6), (2, 3.1e6)])
def test_random_iq_records(gpu, C, fc):
    """Random complex records, three transmit kinds, t0 != 0, ragged grid;
    1 and 3 complex items (pairs in two- and four-item thread groups)."""
    g = _geometry()
    rng = np.random.default_rng(C)
    y = rng.normal(size=(C, g.Q, g.M, g.K)) + 1j * rng.normal(size=(C, g.Q, g.M, g.K))
    y = y.astype(np.complex64)
    x = _run(g, y, fc, gpu)
    _check(x, forward_iq(y, g, fc), f"fc={fc / 1e6} MHz")


def test_zero_carrier_equals_two_real_lanes(gpu):
    """fc = 0: the I and Q outputs equal the real beamformer of each record bit
    for bit (the rotation is the identity)."""
    das = _das()
    g = _geometry()
    y = synth.random_channel_data(g, 2, seed=4)
    p_iq = das.Plan(g, max_batch=2, storage="f32", algo="tiled")
    p_iq.set_iq(0.0)
    p_re = das.Plan(g, max_batch=2, storage="f32", algo="tiled")
    assert torch.equal(p_iq.forward(y.to(gpu)), p_re.forward(y.to(gpu)))


def test_cfg2_block_demodulated_with_transmit_weights(gpu):
    """Simulated cfg2 echoes, made analytic (FFT Hilbert transform) and
    demodulated at 7.5 MHz, on a block around a point target, with
    spatially selective transmit weights (sparse lists in the IQ kernel)."""
    g, y = cfg2_channel_data()
    sub = synth.sub_grid(g, (40, 52, 30), (20, 12, 10))
    ya = metrics.analytic_lanes(y).cpu().numpy().astype(np.float64)
    y_iq = demodulate(ya[0] + 1j * ya[1], g.fs, g.t0, 7.5e6)[None].astype(np.complex64)
    w = synth.selective_tx_weights(sub)
    x = _run(sub, y_iq, 7.5e6, gpu, w_tx=w)
    _check(x, forward_iq(y_iq, sub, 7.5e6, w_tx=w), "cfg2 block")


def test_iq_refusals(gpu):
    das = _das()
    g = _geometry()
    p = das.Plan(g, max_batch=4, storage="f32", algo="tiled")
    p.set_iq(7.5e6)
    with pytest.raises(das.DasError) as e:
        p.forward(synth.random_channel_data(g, 3, seed=1).to(gpu))
    assert e.value.status == das.DAS_ERR_INVALID_ARG
    with pytest.raises(das.DasError) as e:
        p.adjoint(torch.zeros(3, p.N, device=gpu))
    assert e.value.status == das.DAS_ERR_INVALID_ARG
    p16 = das.Plan(g, max_batch=4, storage="f16", algo="tiled")
    p16.set_iq(7.5e6)
    with pytest.raises(das.DasError) as e:
        p16.forward(synth.random_channel_data(g, 2, seed=1).to(gpu))
    assert e.value.status == das.DAS_ERR_UNSUPPORTED
    with pytest.raises(das.DasError) as e:
        p.set_iq(-1.0)
    assert e.value.status == das.DAS_ERR_INVALID_ARG


# --- the transpose of the complex baseband map (oracle.iq.adjoint_iq) ---

def _run_adjoint(g, gx, fc, gpu, w_tx=None):
    """gx complex [C, N] -> GPU gy complex [C, Q, M, K] (I/Q interleaved items)."""
    das = _das()
    C = gx.shape[0]
    lanes = np.empty((2 * C, g.N), np.float32)
    lanes[0::2] = gx.real
    lanes[1::2] = gx.imag
    plan = das.Plan(g, max_batch=2 * C, storage="f32", algo="tiled")
    plan.set_iq(fc)
    if w_tx is not None:
        plan.set_tx_weights(torch.from_numpy(w_tx).to(gpu))
    gy = plan.adjoint(torch.from_numpy(lanes).to(gpu)).cpu().numpy().astype(np.float64)
    return gy[0::2] + 1j * gy[1::2]


@pytest.mark.parametrize("C,fc", [(1, 7.5e6), (2, 3.1e6)])
def test_iq_adjoint_vs_oracle(gpu, C, fc):
    g = _geometry()
    rng = np.random.default_rng(40 + C)
    gx = rng.normal(size=(C, g.N)) + 1j * rng.normal(size=(C, g.N))
    gx = gx.astype(np.complex64)  # the values the GPU receives
    gy = _run_adjoint(g, gx, fc, gpu)
    gyo = adjoint_iq(gx, g, fc)
    for c in range(C):
        check_close(np.concatenate([gy[c].real.ravel(), gy[c].imag.ravel()]),
                    np.concatenate([gyo[c].real.ravel(), gyo[c].imag.ravel()]),
                    REL_L2_F32, ABS_F32, f"IQ adjoint fc={fc / 1e6} MHz item {c}")


def test_iq_adjoint_tx_weights(gpu):
    """Spatially selective transmit weights (about half of each transmit's
    voxels at zero) scaled by random factors."""
    sub = _geometry()
    rng = np.random.default_rng(44)
    w = synth.selective_tx_weights(sub) * rng.uniform(0.2, 1.0, size=(sub.Q, sub.N)).astype(np.float32)
    assert np.count_nonzero(w) > 0
    gx = (rng.normal(size=(1, sub.N)) + 1j * rng.normal(size=(1, sub.N))).astype(np.complex64)
    gy = _run_adjoint(sub, gx, 7.5e6, gpu, w_tx=w)
    gyo = adjoint_iq(gx, sub, 7.5e6, w_tx=w)
    check_close(np.concatenate([gy[0].real.ravel(), gy[0].imag.ravel()]),
                np.concatenate([gyo[0].real.ravel(), gyo[0].imag.ravel()]),
                REL_L2_F32, ABS_F32, "IQ adjoint with transmit weights")


def test_iq_adjoint_dot_product(gpu):
    """<A y, x> = <y, A^T x> in the real inner product over the I/Q lanes,
    both sides through the windowed kernels."""
    das = _das()
    g = _geometry()
    rng = np.random.default_rng(45)
    y = torch.from_numpy(rng.normal(size=(4, g.Q, g.M, g.K)).astype(np.float32)).to(gpu)
    x = torch.from_numpy(rng.normal(size=(4, g.N)).astype(np.float32)).to(gpu)
    plan = das.Plan(g, max_batch=4, storage="f32", algo="tiled")
    plan.set_iq(7.5e6)
    lhs = float((plan.forward(y).double() * x.double()).sum())
    rhs = float((y.double() * plan.adjoint(x).double()).sum())
    say(f"  <Ay,x>={lhs:.9e} <y,A^T x>={rhs:.9e} (IQ)")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("geom", ["small", "cfg5_block"])
def test_iq_grad_sound_speed_vs_oracle(gpu, geom):
    """dL/dc of the complex baseband form (delay and phase both move with c)
    against oracle.iq.grad_sound_speed_iq at the bar of the real form."""
    from oracle.iq import grad_sound_speed_iq
    das = _das()
    g = _geometry() if geom == "small" else synth.sub_grid(synth.cfg5(), (24, 24, 20), (12, 10, 8))
    rng = np.random.default_rng(46)
    C = 2
    y = rng.normal(size=(C, g.Q, g.M, g.K)) + 1j * rng.normal(size=(C, g.Q, g.M, g.K))
    gx = rng.normal(size=(C, g.N)) + 1j * rng.normal(size=(C, g.N))
    y, gx = y.astype(np.complex64), gx.astype(np.complex64)
    ref = grad_sound_speed_iq(y, gx, g, 7.5e6)
    yl = np.empty((2 * C,) + y.shape[1:], np.float32)
    yl[0::2], yl[1::2] = y.real, y.imag
    gl = np.empty((2 * C, g.N), np.float32)
    gl[0::2], gl[1::2] = gx.real, gx.imag
    plan = das.Plan(g, max_batch=2 * C, storage="f32")
    plan.set_iq(7.5e6)
    got = float(plan.grad_sound_speed(torch.from_numpy(yl).to(gpu), torch.from_numpy(gl).to(gpu)))
    say(f"  IQ dL/dc gpu={got:.7e} oracle={ref:.7e}")
    assert abs(got - ref) <= 1e-4 * abs(ref)
    with pytest.raises(das.DasError) as e:
        plan.grad_sound_speed(torch.from_numpy(yl[:3]).to(gpu), torch.from_numpy(gl[:3]).to(gpu))
    assert e.value.status == das.DAS_ERR_INVALID_ARG


# --- complex baseband in the MFMA locality form (Alg. 3 with complex W) ---
# Bars: f16 / FP8 storage of the I and Q records against the oracle on the raw
# complex data (the storage bars of the real forms), and the kernel alone
# against the oracle on the values the workspace holds: the cosine- and
# sine-weighted interpolation weights are f16 (relative rounding 2^-11), as in
# the real MFMA form (5e-4 rel-L2, 1e-3 elementwise).
MFMA_KERNEL = (5e-4, 1e-3)


def _run_mfma(g, y_iq, fc, gpu, storage, form):
    das = _das()
    C = y_iq.shape[0]
    lanes = np.empty((2 * C,) + y_iq.shape[1:], np.float32)
    lanes[0::2] = y_iq.real
    lanes[1::2] = y_iq.imag
    plan = das.Plan(g, max_batch=2 * C, storage=storage, algo="mfma")
    plan.set_iq(fc)
    plan.set_mfma_form(form)
    x = plan.forward(torch.from_numpy(lanes).to(gpu)).cpu().numpy().astype(np.float64)
    return x[0::2] + 1j * x[1::2], lanes


def _check_c(x, xo, rel, absf, what):
    for c in range(x.shape[0]):
        check_close(np.concatenate([x[c].real, x[c].imag]), np.concatenate([xo[c].real, xo[c].imag]),
                    rel, absf, f"{what} item {c}")


@pytest.mark.parametrize("form", ["column", "slab"])
@pytest.mark.parametrize("storage", ["f16", "fp8"])
@pytest.mark.parametrize("C", [8, 17, 32])
def test_iq_mfma_random_records(gpu, form, storage, C):
    """Random complex records, three transmit kinds, t0 != 0, ragged grid;
    16, 34 and 64 batch columns (one tile, a ragged pair of 64-column tiles
    covered in halves, two full tiles)."""
    from tests.gpu_util import lowp_bars, round_like_storage
    g = _geometry()
    rng = np.random.default_rng(100 + C)
    y = (rng.normal(size=(C, g.Q, g.M, g.K)) + 1j * rng.normal(size=(C, g.Q, g.M, g.K))).astype(np.complex64)
    say(f"IQ mfma {form} {storage}, {C} complex items")
    x, lanes = _run_mfma(g, y, 7.5e6, gpu, storage, form)
    items = sorted({0, C // 2, C - 1})
    _check_c(x[items], forward_iq(y[items], g, 7.5e6), *lowp_bars(storage), "raw data")
    r = round_like_storage(lanes, storage)
    yr = r[0::2] + 1j * r[1::2]
    _check_c(x[items], forward_iq(yr[items], g, 7.5e6), *MFMA_KERNEL, "  rounded data")


@pytest.mark.parametrize("storage", ["f16", "fp8"])
@pytest.mark.parametrize("C", [8, 17])
def test_iq_mfma_persistent_form(gpu, storage, C):
    """The persistent kernel's complex baseband body: the column launch (the
    same wavefront boxes and batch tiles per wavefront) bit for bit, and the
    oracle at the storage bars."""
    from tests.gpu_util import lowp_bars
    g = _geometry()
    rng = np.random.default_rng(200 + C)
    y = (rng.normal(size=(C, g.Q, g.M, g.K)) + 1j * rng.normal(size=(C, g.Q, g.M, g.K))).astype(np.complex64)
    say(f"IQ mfma persistent {storage}, {C} complex items")
    x, _ = _run_mfma(g, y, 7.5e6, gpu, storage, "persistent")
    xc, _ = _run_mfma(g, y, 7.5e6, gpu, storage, "column")
    assert np.array_equal(x, xc), "persistent IQ launch differs from the column launch"
    items = sorted({0, C - 1})
    _check_c(x[items], forward_iq(y[items], g, 7.5e6), *lowp_bars(storage), "persistent")


def test_iq_mfma_batched_launch(gpu):
    """One persistent launch over two complex baseband plans (different grids,
    arrays, transmit counts and batch sizes) equals separate persistent
    launches bit for bit and the oracle within the f16 bars; a launch that
    mixes complex and real plans, an odd complex batch and windowed complex
    plans are refused."""
    from tests.gpu_util import lowp_bars
    das = _das()
    geoms = [_geometry(), synth.sub_grid(synth.cfg5(), (20, 24, 10), (9, 8, 12))]
    counts = [8, 9]
    plans, wss, xs, ys = [], [], [], []
    for i, (g, C) in enumerate(zip(geoms, counts)):
        rng = np.random.default_rng(300 + i)
        y = (rng.normal(size=(C, g.Q, g.M, g.K)) + 1j * rng.normal(size=(C, g.Q, g.M, g.K))).astype(np.complex64)
        lanes = np.empty((2 * C,) + y.shape[1:], np.float32)
        lanes[0::2], lanes[1::2] = y.real, y.imag
        p = das.Plan(g, max_batch=2 * C, storage="f16", algo="mfma")
        p.set_iq(7.5e6)
        wss.append(p.prepare(torch.from_numpy(lanes).to(gpu)))
        plans.append(p)
        xs.append(torch.full((2 * C, p.N), float("nan"), device=gpu))
        ys.append(y)
    batches = [2 * C for C in counts]
    das.das_forward_batched([p.handle for p in plans], wss, batches, xs)
    for p, ws, x, y, g, B in zip(plans, wss, xs, ys, geoms, batches):
        p.set_mfma_form("persistent")
        assert torch.equal(x, p.forward_ws(ws, B)), "batched IQ launch differs from a separate launch"
        xn = x.cpu().numpy().astype(np.float64)
        xc = xn[0::2] + 1j * xn[1::2]
        items = [0, B // 2 - 1]
        _check_c(xc[items], forward_iq(y[items], g, 7.5e6), *lowp_bars("f16"), f"batched IQ {g.grid_dims}")
    # a real plan cannot join a complex launch
    g = geoms[0]
    p_r = das.Plan(g, max_batch=16, storage="f16", algo="mfma")
    ws_r = p_r.prepare(synth.random_channel_data(g, 16, seed=4).to(gpu))
    with pytest.raises(das.DasError) as e:
        das.das_forward_batched([plans[0].handle, p_r.handle], [wss[0], ws_r], [16, 16],
                                [xs[0], torch.empty(16, p_r.N, device=gpu)])
    assert e.value.status == das.DAS_ERR_UNSUPPORTED
    # odd complex batch
    with pytest.raises(das.DasError) as e:
        das.das_forward_batched([plans[1].handle], [wss[1]], [17], [xs[1]])
    assert e.value.status == das.DAS_ERR_INVALID_ARG
    # windowed complex plans run through das_forward only
    p_w = das.Plan(g, max_batch=2, storage="f32", algo="tiled")
    p_w.set_iq(7.5e6)
    ws_w = p_w.prepare(synth.random_channel_data(g, 2, seed=5).to(gpu))
    with pytest.raises(das.DasError) as e:
        das.das_forward_batched([p_w.handle], [ws_w], [2], [torch.empty(2, p_w.N, device=gpu)])
    assert e.value.status == das.DAS_ERR_UNSUPPORTED


def test_iq_mfma_refuses_bf16(gpu):
    das = _das()
    g = _geometry()
    p = das.Plan(g, max_batch=16, storage="bf16", algo="mfma")
    p.set_iq(7.5e6)
    with pytest.raises(das.DasError) as e:
        p.forward(synth.random_channel_data(g, 16, seed=2).to(gpu))
    assert e.value.status == das.DAS_ERR_UNSUPPORTED


def test_iq_cfg2_full_volume_sampled(gpu):
    """The full 128^3 x 1024 x 16 volume in complex baseband, as the benchmark
    forms run it: the simulated cfg2 frame made analytic and demodulated at
    7.5 MHz, one complex frame through the windowed FP32 kernel, and the same
    frame repeated 8 times through the MFMA form (f16 storage, column launch);
    sampled voxels against the oracle computed one by one."""
    from tests.gpu_util import lowp_bars, sample_voxels
    das = _das()
    g, y = cfg2_channel_data()
    za = metrics.analytic_lanes(y)
    tk = g.t0 + torch.arange(g.K, device=y.device, dtype=torch.float64) / g.fs
    ph = -2.0 * np.pi * 7.5e6 * tk
    lanes = torch.stack([za[0] * torch.cos(ph).float() - za[1] * torch.sin(ph).float(),
                         za[0] * torch.sin(ph).float() + za[1] * torch.cos(ph).float()]).contiguous()
    del za
    idx = sample_voxels(g, 384, seed=11)
    ln = lanes.cpu().numpy()
    xo = forward_iq((ln[0] + 1j * ln[1])[None], g, 7.5e6, voxels=idx)[0]
    ref = np.concatenate([xo.real, xo.imag])

    plan = das.Plan(g, max_batch=2, storage="f32", algo="tiled")
    plan.set_iq(7.5e6)
    x = plan.forward(lanes).cpu().numpy().astype(np.float64)
    check_close(np.concatenate([x[0][idx], x[1][idx]]), ref, REL_L2_F32, ABS_F32,
                "IQ cfg2 full, windowed FP32, sampled voxels")
    plan.close()

    p16 = das.Plan(g, max_batch=16, storage="f16", algo="mfma")
    p16.set_iq(7.5e6)
    p16.set_mfma_form("column")
    x8 = p16.forward(lanes.repeat(8, 1, 1, 1).contiguous()).cpu().numpy().astype(np.float64)
    for c in (0, 7):
        check_close(np.concatenate([x8[2 * c][idx], x8[2 * c + 1][idx]]), ref, *lowp_bars("f16"),
                    f"IQ cfg2 full, MFMA f16 column, complex item {c}, sampled voxels")
    p16.close()


def test_iq_adjoint_cfg5_full_size_sampled_channels(gpu):
    """The complex baseband adjoint at the full differentiable-case size
    (64^3 voxels, 16x16 array, 8 plane waves, one (I, Q) pair) in the launch
    the benchmark times, checked on sampled channels: the oracle's adjoint_iq
    of a geometry that holds only the sampled elements gives those elements'
    rows for every transmit."""
    das = _das()
    g = synth.cfg5()
    rng = np.random.default_rng(12)
    gx = (rng.normal(size=(1, g.N)) + 1j * rng.normal(size=(1, g.N))).astype(np.complex64)
    lanes = np.empty((2, g.N), np.float32)
    lanes[0], lanes[1] = gx.real[0], gx.imag[0]
    plan = das.Plan(g, max_batch=2, storage="f32")
    plan.set_iq(7.5e6)
    say(f"IQ adjoint cfg5 full size {g.grid_dims} x {g.M} el x {g.Q} tx")
    gy = plan.adjoint(torch.from_numpy(lanes).to(gpu)).cpu().numpy().astype(np.float64)
    sel = np.sort(rng.choice(g.M, size=6, replace=False))
    sel = np.unique(np.concatenate([sel, [0, g.M - 1]]))
    sub = g.replace(elem_pos=np.asarray(g.elem_pos)[sel],
                    elem_normal=None if g.elem_normal is None else np.asarray(g.elem_normal)[sel])
    gyo = adjoint_iq(gx, sub, 7.5e6)[0]
    got = gy[0][:, sel] + 1j * gy[1][:, sel]
    check_close(np.concatenate([got.real.ravel(), got.imag.ravel()]),
                np.concatenate([gyo.real.ravel(), gyo.imag.ravel()]), REL_L2_F32, ABS_F32,
                f"IQ adjoint cfg5, elements {sel.tolist()}")

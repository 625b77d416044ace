#!/usr/bin/env python3
"""Volumes/s of the 3D delay-and-sum hot path on one MI355X.

Workload (default): 128^3 voxels x 1024 elements (32x32 matrix array) x 16
diverging-wave transmits, K = 2048 samples, Hann receive apodization F = 1.5,
one frame per step, FP32.  A step is one pass of the whole hot path over one
batch: reorder + convert (das_prepare) then the forward kernel (das_forward),
with the channel data already resident in HBM.  Other forms (FP16 / BF16
storage, the matrix-core form, batched frames and a 256-frame ensemble) are
measured after the headline and reported under "forms".

Prints ONE JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("volumes/s at 128³ vox×1024 el×16 tx: FP32 vs FP16/MFMA at stated L2 error")
# MI355X published peaks: FP32 vector 157.3 TFLOP/s (packed FMA), dense FP16
# MFMA 2.5 PFLOP/s, HBM3E 8 TB/s.  Packed-FP32 instructions are not generated
# by this build, so the kernels' own VALU ceiling is the non-packed rate:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane operations/s, 78.6
# TFLOP/s counting an FMA as 2 flops; it is reported beside the published peak.
VALU_PEAK_TFLOPS = 157.3
VALU_NONPACKED_TFLOPS = 256 * 4 * 16 * 2.4e9 * 2 / 1e12
MFMA_F16_PEAK_TFLOPS = 2500.0
HBM_PEAK_GBS = 8000.0
# Algorithmic work model (flops): 25 per nonzero (voxel, element) pair (receive
# path and apodization), 12 per nonzero (pair, transmit) triple (index and
# weight formation), 4 per (triple, batch item) (two taps: 2 FMAs).
FLOPS_PER_PAIR, FLOPS_PER_TRIPLE, FLOPS_PER_ITEM = 25, 12, 4
STORAGE_BYTES = {"f32": 4, "f16": 2, "bf16": 2, "fp8": 1}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def work_counts(name):
    with open(os.path.join(ROOT, "tests", "golden", "nonzero_counts.json")) as f:
        return json.load(f)[name]


def algorithmic_flops(counts, batch):
    return (FLOPS_PER_PAIR * counts["pairs_nonzero"] + FLOPS_PER_TRIPLE * counts["triples_nonzero"]
            + FLOPS_PER_ITEM * counts["triples_nonzero"] * batch)


def valu_roofline(flops, ms, kernel=None, traffic=None):
    """Algorithmic flops per launch over the launch's mean duration, against
    the published FP32 peak, with the non-packed ceiling beside it."""
    achieved = flops / (ms * 1e-3) / 1e12
    out = {"bound": "alu", "achieved": round(achieved, 3), "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": round(achieved / VALU_PEAK_TFLOPS, 4), "traffic": traffic,
           "nonpacked_peak": round(VALU_NONPACKED_TFLOPS, 1),
           "frac_nonpacked": round(achieved / VALU_NONPACKED_TFLOPS, 4),
           "kernel_ms": round(ms, 4), "flops_per_launch": int(flops)}
    if kernel:
        out["kernel"] = kernel
    return out


def mfma_roofline(counts, B, storage, g, ms, traffic=None, kernel=None):
    """The matrix-core form: useful flops (2 MACs per nonzero triple and item)
    against the dense FP16 MFMA peak, and algorithmic bytes (the stored
    samples of every item in, the f32 volume out) against HBM."""
    flops = FLOPS_PER_ITEM * counts["triples_nonzero"] * B
    nbytes = B * (g.Q * g.M * g.K * STORAGE_BYTES[storage] + 4 * g.N)
    t = ms * 1e-3
    out = {"bound": "mfma", "achieved": round(flops / t / 1e12, 3), "peak": MFMA_F16_PEAK_TFLOPS,
           "unit": "TFLOP/s", "frac": round(flops / t / 1e12 / MFMA_F16_PEAK_TFLOPS, 5),
           "traffic": traffic, "kernel_ms": round(ms, 4), "useful_flops_per_launch": int(flops),
           "hbm": {"achieved": round(nbytes / t / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4),
                   "algorithmic_bytes_per_launch": int(nbytes)}}
    if traffic:
        out["traffic_over_algorithmic"] = round(traffic / nbytes, 2)
    if kernel:
        out["kernel"] = kernel
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def recorded_traffic(kernel, tile):
    """HBM traffic per launch of `kernel` from the rocprofv3 FETCH_SIZE / WRITE_SIZE
    passes recorded in profiles/traffic.json (each scaled by what the counter reads
    for a plain copy of known size), or None when the kernel's sources have changed
    since the counters were taken or they were taken with another tile shape (for
    the matrix-core form: another launch form)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)[kernel]
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
    except (OSError, KeyError, ValueError):
        return None
    if h.hexdigest() != rec["sources_sha256"] or list(rec["tile"]) != list(tile):
        return None
    return rec["traffic_bytes_per_launch"]


def time_form(torch, das, plan, y, steps, warmup):
    """Time `steps` (prepare + forward) steps; returns wall ms/step and the
    mean duration of each of the two kernels from HIP events on the stream
    they run on."""
    B = y.shape[0]
    stream = torch.cuda.current_stream()
    ws = plan.workspace(B)
    x = torch.empty(B, plan.N, dtype=torch.float32, device=y.device)
    for _ in range(warmup):
        das.das_prepare(plan.handle, y, 0, B, B, ws)
        das.das_forward(plan.handle, ws, B, x)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        das.das_prepare(plan.handle, y, 0, B, B, ws)
        ev[i][1].record(stream)
        das.das_forward(plan.handle, ws, B, x)
        ev[i][2].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    prep = sum(e[0].elapsed_time(e[1]) for e in ev) / steps
    fwd = sum(e[1].elapsed_time(e[2]) for e in ev) / steps
    time_form.last_steps = [e[0].elapsed_time(e[2]) for e in ev]  # per-step device time
    return wall, prep, fwd, x


def oracle_sample(oracle, y_np, g, idx, workers):
    """The FP64 oracle on the voxels idx of every item of y_np (process pool)."""
    xo, used = oracle.forward_slabs_parallel(y_np, g, voxels=idx, workers=workers, chunk=512)
    return xo, used


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=1 << 20,
                    help="voxels of the volume the CPU oracle evaluates (default: half the volume)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="f16,bf16,fp8",
                    help="extra storage forms to time after the FP32 headline ('' for none)")
    ap.add_argument("--plain", default="1,8",
                    help="batch sizes of the plain FP32 kernel forms ('' for none)")
    ap.add_argument("--batched", type=int, default=16,
                    help="frames per step for the batched form (0 = skip)")
    ap.add_argument("--ensemble", type=int, default=256,
                    help="frames of the Doppler ensemble (motion frames; 0 = skip)")
    ap.add_argument("--ensemble-data", choices=("motion", "repeat"), default="motion",
                    help="ensemble frames: simulated motion frames, or the cfg2 frame repeated "
                         "(profiling runs: the timing does not depend on the values)")
    ap.add_argument("--ensemble-storage", default="f16,fp8",
                    help="storage types of the ensemble MFMA forms")
    ap.add_argument("--no-ensemble-extras", dest="ensemble_extras", action="store_false",
                    help="skip the persistent mixed launches, the Doppler pipeline and the clutter filter")
    ap.add_argument("--no-adjoint", dest="adjoint", action="store_false",
                    help="skip timing the adjoint and sound-speed gradient (cfg5)")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-sparse-tx", dest="sparse_tx", action="store_false",
                    help="skip the spatially selective transmit-weight forms")
    ap.add_argument("--no-iq", dest="iq", action="store_false", help="skip the complex baseband forms")
    ap.add_argument("--no-cubic", dest="cubic", action="store_false",
                    help="skip the cubic-interpolation form")
    ap.add_argument("--tile", type=int, default=None,
                    help="use this tile shape index instead of autotuning (profiling runs)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(frames or voxel slabs would shard with no communication)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2606_13259_amd import das

    dev = torch.device("cuda:0")
    das.lib()
    t_sim = time.perf_counter()
    log("simulating cfg2 channel data on the GPU")
    g, _, yq = synth.cfg2_data(device="cuda:0")
    y = yq[None].contiguous()
    torch.cuda.synchronize()
    log(f"  simulated in {time.perf_counter() - t_sim:.1f} s")
    counts = work_counts("cfg2")

    plan = das.Plan(g, max_batch=max(1, args.batched), storage="f32")
    if args.tile is not None:
        plan.set_tile(args.tile)
    elif not args.no_autotune:
        t = plan.autotune(1)
        log(f"autotuned tile {das.das_tile_shape(t)}")
    log(f"algo={plan.algo(1)} tile={das.das_tile_shape(plan.tile())}")
    wall, prep_ms, fwd_ms, x = time_form(torch, das, plan, y, args.steps, args.warmup)
    st_ms = np.sort(np.asarray(time_form.last_steps))
    step_pct = {"p10": round(float(np.percentile(st_ms, 10)), 4),
                "median": round(float(np.median(st_ms)), 4),
                "p90": round(float(np.percentile(st_ms, 90)), 4), "unit": "ms (prepare + forward, HIP events)"}
    value = 1000.0 / wall
    log(f"FP32: {wall:.3f} ms/step (prepare {prep_ms:.3f} ms, forward {fwd_ms:.3f} ms) -> {value:.1f} volumes/s")

    kernel = "tiled_forward<float,1,16,false>"
    tile = list(das.das_tile_shape(plan.tile()))
    roofline = valu_roofline(algorithmic_flops(counts, 1), fwd_ms, kernel, recorded_traffic(kernel, tile))
    roofline["traffic_unit"] = "bytes per launch"
    prep_bytes = 2 * 4 * g.Q * g.M * g.K
    reorder = {"bound": "hbm", "achieved": round(prep_bytes / (prep_ms * 1e-3) / 1e9, 1),
               "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(prep_bytes / (prep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "kernel_ms": round(prep_ms, 4)}

    # --- oracle on a bounded sample of voxels: stated L2 error + CPU baseline
    rng = np.random.default_rng(1234)
    idx = np.sort(rng.choice(g.N, size=min(args.cpu_sample, g.N), replace=False))
    idx_t = torch.from_numpy(idx).to(dev)
    xs = {"f32_b1": x[0, idx_t].cpu().numpy()}
    cpu_baseline = None
    xo = None
    workers = min(16, os.cpu_count() or 1)
    if not args.no_cpu_baseline:
        import oracle
        log(f"oracle: {idx.size} voxels x {g.M} elements x {g.Q} transmits on {workers} processes")
        yc = y.cpu().numpy()
        t0 = time.perf_counter()
        xo, used = oracle_sample(oracle, yc, g, idx, workers)
        t_cpu = time.perf_counter() - t0
        xo = xo[0]
        per_volume = t_cpu * g.N / idx.size
        cpu_baseline = {"value": round(1.0 / per_volume, 6), "unit": "volumes/s", "cores": used,
                        "kind": "oracle", "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
                        "sample": f"{idx.size} random voxels ({idx.size / g.N:.3f} of the 128^3 "
                                  f"volume), all 1024 elements x 16 transmits (FP64 NumPy, process "
                                  f"pool of {used}); {t_cpu:.1f} s wall, scaled by N/sample"}
        log(f"oracle: {t_cpu:.1f} s -> {1.0 / per_volume:.2e} volumes/s")

    def rel(v, ref=None):
        ref = xo if ref is None else ref
        if ref is None:
            return None
        return float(np.linalg.norm(v - ref) / np.linalg.norm(ref))

    forms = {}

    def run_form(name, storage, algo, yb, steps, note=None, w_tx=None, iq_fc=None, roof=None,
                 check=True, interp=None, mfma_form=None):
        B = yb.shape[0]
        pf = das.Plan(g, max_batch=B, storage=storage, algo=algo)
        if interp is not None:
            pf.set_interp(interp)
        if w_tx is not None:
            pf.set_tx_weights(w_tx)
        if iq_fc is not None:
            pf.set_iq(iq_fc)
        if pf.algo(B) == "tiled":
            pf.set_tile(plan.tile())
        elif mfma_form is not None:
            pf.set_mfma_form(mfma_form)
        elif pf.algo(B) == "mfma":
            pf.autotune(B)
        wf, prf, fwf, xf = time_form(torch, das, pf, yb, steps, 1)
        f = {"volumes_per_s": round(1000.0 * B / wf, 2), "ms_per_step": round(wf, 4),
             "forward_ms": round(fwf, 4), "prepare_ms": round(prf, 4), "batch": B,
             "storage": storage, "algo": pf.algo(B),
             "mfma_form": pf.mfma_form() if pf.algo(B) == "mfma" else None,
             "rel_l2": rel(xf[0, idx_t].cpu().numpy()) if check else None}
        if roof == "valu":
            f["roofline"] = valu_roofline(algorithmic_flops(counts, B), fwf)
        elif roof == "mfma":
            f["roofline"] = mfma_roofline(counts, B, storage, g, fwf)
        if note:
            f["data"] = note
        forms[name] = f
        log(f"{name}: {wf:.3f} ms/step (forward {fwf:.3f} ms) -> {1000.0 * B / wf:.1f} volumes/s "
            f"[{pf.algo(B)}]")
        pf.close()
        return xf

    for st in [s for s in args.forms.split(",") if s]:
        del_x = run_form(f"{st}_b1", st, "auto", y, max(3, args.steps // 2), roof="valu")
        del del_x
    # The plain kernel (per-voxel gathers from the caller's layout, no window
    # staging, no aperture culling): the baseline of the windowed kernel.
    for pb in [int(s) for s in args.plain.split(",") if s]:
        yb = y.expand(pb, -1, -1, -1).contiguous() if pb > 1 else y
        del_x = run_form(f"f32_plain_b{pb}", "f32", "plain", yb, 3, roof="valu",
                         note=None if pb == 1 else "the simulated frame repeated")
        del del_x, yb
    # Four-point Lagrange (cubic) interpolation instead of the linear taps of
    # Eq. (2), the windowed FP32 kernel (its oracle parity is in the GPU tests).
    if args.cubic:
        del_x = run_form("f32_cubic_b1", "f32", "tiled", y, max(3, args.steps // 2), check=False,
                         interp="cubic", note="cubic interpolation of the simulated frame")
        del del_x
    if args.sparse_tx:
        # A spatially selective transmit sequence (each transmit weighs one
        # lateral cell of a 4 x 4 layout, widened and tapered, zero elsewhere):
        # per-tile sparse transmit lists against the same weights with the
        # zeros raised to 1e-30 (every transmit live everywhere).
        wsel = torch.from_numpy(synth.selective_tx_weights(g)).to(dev)
        note = (f"transmit weights: spatially selective, {float((wsel > 0).float().mean()):.3f} of "
                f"(transmit, voxel) pairs nonzero")
        run_form("f32_b1_tx_weights_all_live", "f32", "auto", y, max(3, args.steps // 2), note=note,
                 w_tx=wsel.clamp_min(1e-30).contiguous(), check=False)
        run_form("f32_b1_tx_weights_sparse", "f32", "auto", y, max(3, args.steps // 2), note=note,
                 w_tx=wsel, check=False)
        del wsel
    if args.iq:
        # Complex baseband: the simulated frame made analytic and demodulated at
        # 7.5 MHz, one complex volume per step as an (I, Q) pair.
        from paper_2606_13259_amd import metrics
        za = metrics.analytic_lanes(y[0])
        tk = g.t0 + torch.arange(g.K, device=dev, dtype=torch.float64) / g.fs
        ph = -2.0 * np.pi * 7.5e6 * tk
        yiq = torch.stack([za[0] * torch.cos(ph).float() - za[1] * torch.sin(ph).float(),
                           za[0] * torch.sin(ph).float() + za[1] * torch.cos(ph).float()]).contiguous()
        run_form("f32_iq_b1", "f32", "tiled", yiq, max(3, args.steps // 2), iq_fc=7.5e6, check=False,
                 note="IQ: the simulated frame, analytic and demodulated at 7.5 MHz; one complex volume "
                      "per step (batch = the I and Q records)")
        forms["f32_iq_b1"]["volumes_per_s"] = round(forms["f32_iq_b1"]["volumes_per_s"] / 2, 2)
        forms["f32_iq_b1"]["unit_note"] = "complex volumes/s"
        # the same complex frame, 8 times, on the matrix cores (f16 storage,
        # the launch form the autotuner picks)
        yiq8 = yiq.repeat(8, 1, 1, 1).contiguous()
        run_form("f16_iq_mfma_b16", "f16", "mfma", yiq8, max(2, args.steps // 4), iq_fc=7.5e6,
                 check=False,
                 note="IQ: the demodulated frame repeated; 8 complex volumes per step (16 items)")
        forms["f16_iq_mfma_b16"]["volumes_per_s"] = round(forms["f16_iq_mfma_b16"]["volumes_per_s"] / 2, 2)
        forms["f16_iq_mfma_b16"]["unit_note"] = "complex volumes/s"
        del za, yiq, yiq8
    if args.batched > 1:
        B = args.batched
        yb = y.expand(B, -1, -1, -1).contiguous()
        steps = max(2, args.steps // 4)
        note = "the simulated frame repeated"
        for name, st, algo, roof in ((f"f32_tiled_b{B}", "f32", "tiled", "valu"),
                                     (f"f16_tiled_b{B}", "f16", "tiled", "valu"),
                                     (f"f16_mfma_b{B}", "f16", "mfma", "mfma"),
                                     (f"bf16_mfma_b{B}", "bf16", "mfma", "mfma"),
                                     (f"fp8_mfma_b{B}", "fp8", "mfma", "mfma")):
            del_x = run_form(name, st, algo, yb, steps, roof=roof, note=note)
            del del_x
        del yb
    torch.cuda.empty_cache()
    if args.ensemble > 1:
        run_ensemble(args, torch, np, das, synth, g, counts, forms, workers)
    torch.cuda.empty_cache()

    if args.adjoint:
        # The differentiable form (cfg5 geometry: 64^3, 16x16 array, 8 plane waves, FP32,
        # Re and Im lanes): forward, adjoint (channel-data gradient) and dL/dc;
        # also the adjoint and dL/dc of the complex baseband form (the two
        # lanes as one (I, Q) pair demodulated at 7.5 MHz).
        g5 = synth.cfg5()
        p5 = das.Plan(g5, max_batch=2, storage="f32")
        p5q = das.Plan(g5, max_batch=2, storage="f32")
        p5q.set_iq(7.5e6)
        torch.manual_seed(5)
        y5 = torch.randn(2, g5.Q, g5.M, g5.K, device=dev)
        gx = torch.randn(2, p5.N, device=dev)
        ws5 = p5.prepare(y5)
        x5 = p5.forward_ws(ws5, 2)
        gy = p5.adjoint(gx)
        gyq = p5q.adjoint(gx)
        dc = p5.grad_sound_speed(y5, gx)
        reps = max(3, args.steps // 2)
        timings = {}
        for name, fn in (("forward_ms", lambda: p5.forward_ws(ws5, 2, x5)),
                         ("adjoint_ms", lambda: das.das_adjoint(p5.handle, gx, 2, gy)),
                         ("adjoint_iq_ms", lambda: das.das_adjoint(p5q.handle, gx, 2, gyq)),
                         ("grad_c_ms", lambda: p5.grad_sound_speed(y5, gx)),
                         ("grad_c_iq_ms", lambda: p5q.grad_sound_speed(y5, gx))):
            fn()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            timings[name] = round(e0.elapsed_time(e1) / reps, 4)
        forms["cfg5_differentiable"] = dict(timings, batch=2, storage="f32",
                                            workload="64^3 voxels x 256 elements x 8 plane waves",
                                            data="random N(0,1) channel data and upstream gradient")
        log(f"cfg5 forward {timings['forward_ms']:.3f} ms, adjoint {timings['adjoint_ms']:.3f} ms, "
            f"IQ adjoint {timings['adjoint_iq_ms']:.3f} ms, dL/dc {timings['grad_c_ms']:.3f} ms, "
            f"IQ dL/dc {timings['grad_c_iq_ms']:.3f} ms")
        del y5, gx, ws5, x5, gy, gyq, dc
        p5.close()
        p5q.close()

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "volumes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic: 200 point targets + 1e4 speckle scatterers, seeded, ray-model echoes",
        "config": {"workload": "128^3 voxels x 1024 elements (32x32, pitch 0.3 mm) x 16 diverging "
                               "transmits, K=2048, Hann F=1.5, 1 frame per step",
                   "batch": 1, "storage": "f32", "algo": plan.algo(1),
                   "tile": list(das.das_tile_shape(plan.tile()))},
        "rel_l2": rel(xs["f32_b1"]),
        "rel_l2_sample_voxels": int(idx.size),
        "roofline": roofline,
        "reorder_roofline": reorder,
        "cpu_baseline": cpu_baseline,
        "forms": forms,
        "prepare_ms": round(prep_ms, 4), "forward_ms": round(fwd_ms, 4),
        "step_ms_percentiles": step_pct,
        "dense_updates_per_s": round(g.N * g.M * g.Q / (wall * 1e-3), 1),
    }
    print(json.dumps(out), flush=True)


def run_ensemble(args, torch, np, das, synth, g, counts, forms, workers):
    """The Doppler ensemble: 256 frames whose scatterers move by a seeded
    sub-wavelength random walk per frame, beamformed by the MFMA form (f16 and
    FP8 storage), then alone and with the mixed grids in one persistent
    launch, and finally through the clutter filter and power Doppler."""
    import oracle
    dev = torch.device("cuda:0")
    B = args.ensemble
    t0 = time.perf_counter()
    if args.ensemble_data == "repeat":
        _, _, y1 = synth.cfg2_data(device=dev)
        ye = y1[None].expand(B, -1, -1, -1).contiguous()
        del y1
        note = "the cfg2 frame repeated"
    else:
        log(f"simulating {B} motion frames on the GPU")
        _, ye, _ = synth.cfg4_ensemble(B, device=dev, dtype=torch.float32, progress=lambda d, n: log(
            f"  {d}/{n} frames ({time.perf_counter() - t0:.1f} s)"))
        note = ("motion ensemble: the 200 targets + 1e4 speckle scatterers moved by a random walk "
                "N(0, (lambda/40)^2) per axis per frame (seed 5 + frame), simulated in FP32")
    torch.cuda.synchronize()
    log(f"  ensemble ready in {time.perf_counter() - t0:.1f} s")
    check = sorted({0, 1, B // 2, B - 1})
    idx = np.sort(np.random.default_rng(99).choice(g.N, size=2048, replace=False))
    idx_t = torch.from_numpy(idx).to(dev)
    xo = None
    if not args.no_cpu_baseline:
        xo, _ = oracle_sample(oracle, ye[check].cpu().numpy(), g, idx, workers)
    for st in [v for v in args.ensemble_storage.split(",") if v]:
        pf = das.Plan(g, max_batch=B, storage=st)
        pf.autotune(B)  # MFMA launch form picked by timing
        wf, prf, fwf, xf = time_form(torch, das, pf, ye, max(2, args.steps // 8), 1)
        f = {"volumes_per_s": round(1000.0 * B / wf, 2), "ms_per_step": round(wf, 4),
             "forward_ms": round(fwf, 4), "prepare_ms": round(prf, 4), "batch": B, "storage": st,
             "algo": pf.algo(B), "mfma_form": pf.mfma_form(), "per_frame_latency_ms": round(wf, 3),
             "data": note,
             "roofline": mfma_roofline(counts, B, st, g, fwf,
                                       recorded_traffic(f"mfma_forward {st} B={B}", [pf.mfma_form()]))}
        if xo is not None:
            xs = xf[check][:, idx_t].cpu().numpy()
            f["rel_l2_frames"] = {str(fr): float(np.linalg.norm(xs[i] - xo[i]) / np.linalg.norm(xo[i]))
                                  for i, fr in enumerate(check)}
            f["rel_l2_sample_voxels"] = int(idx.size)
        forms[f"{st}_mfma_b{B}"] = f
        log(f"{st}_mfma_b{B}: {wf:.2f} ms/step (forward {fwf:.2f} ms) -> {1000.0 * B / wf:.1f} volumes/s "
            f"[{pf.algo(B)}] rel-L2 {f.get('rel_l2_frames')}")
        pf.close()
        del xf
    torch.cuda.empty_cache()

    # The ensemble plus a mixed batch of grids and arrays in ONE persistent launch.
    def run_persistent(name, storage):
        mixed = synth.mixed_geometries()
        mb = 16
        plans = [das.Plan(g, max_batch=B, storage=storage)]
        wss = [plans[0].prepare(ye)]
        batches = [B]
        for gm in mixed:
            pm = das.Plan(gm, max_batch=mb, storage=storage)
            torch.manual_seed(70)
            wss.append(pm.prepare(torch.randn(mb, gm.Q, gm.M, gm.K, device=dev)))
            plans.append(pm)
            batches.append(mb)
        outs = [torch.empty(b, p.N, dtype=torch.float32, device=dev) for p, b in zip(plans, batches)]
        handles = [p.handle for p in plans]
        das.das_forward_batched(handles, wss, batches, outs)
        stream = torch.cuda.current_stream()
        reps = max(2, args.steps // 8)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            das.das_forward_batched(handles, wss, batches, outs)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        nvol = sum(batches)
        forms[name] = {
            "volumes_per_s": round(1000.0 * nvol / ms, 2), "launch_ms": round(ms, 3),
            "volumes_per_launch": nvol, "storage": storage, "algo": plans[0].algo(B),
            "plans": [{"grid": list(p.geom.grid_dims), "elements": p.M, "batch": b}
                      for p, b in zip(plans, batches)],
            "latency_note": "every frame of a launch completes when the launch does: per-frame "
                            "latency = launch_ms",
            "data": "ensemble: the motion frames; mixed grids: random N(0,1) data"}
        log(f"{name}: {ms:.2f} ms per launch, {nvol} volumes -> {1000.0 * nvol / ms:.1f} volumes/s")
        del wss, outs
        for p in plans:
            p.close()
        torch.cuda.empty_cache()

    if not args.ensemble_extras:
        del ye
        return
    run_persistent("persistent_ensemble_mixed", "f16")
    run_persistent("persistent_ensemble_mixed_fp8", "fp8")

    # End to end: reorder + beamform the motion frames (f16 MFMA), then the
    # rank-truncation clutter filter (3 tissue components removed) and power
    # Doppler over the 256 volumes.
    pf = das.Plan(g, max_batch=B, storage="f16")
    pf.autotune(B)
    ws = pf.workspace(B)
    xe = torch.empty(B, g.N, dtype=torch.float32, device=dev)
    wsc = torch.empty(das.das_clutter_workspace_bytes(B), dtype=torch.uint8, device=dev)
    svc = torch.empty(B, device=dev)
    pwc = torch.empty(g.N, device=dev)

    def pipeline():
        das.das_prepare(pf.handle, ye, 0, B, B, ws)
        das.das_forward(pf.handle, ws, B, xe)
        das.das_clutter_filter(xe, 3, B, svc, pwc, None, wsc)

    pipeline()
    reps = max(2, args.steps // 8)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(reps)]
    torch.cuda.synchronize()
    for i in range(reps):
        ev[i][0].record()
        das.das_prepare(pf.handle, ye, 0, B, B, ws)
        ev[i][1].record()
        das.das_forward(pf.handle, ws, B, xe)
        ev[i][2].record()
        das.das_clutter_filter(xe, 3, B, svc, pwc, None, wsc)
        ev[i][3].record()
    torch.cuda.synchronize()
    part = [sum(e[j].elapsed_time(e[j + 1]) for e in ev) / reps for j in range(3)]
    tot = sum(part)
    forms["doppler_pipeline"] = {
        "frames": B, "voxels": int(g.N), "storage": "f16", "algo": pf.algo(B),
        "prepare_ms": round(part[0], 3), "forward_ms": round(part[1], 3),
        "clutter_filter_ms": round(part[2], 3), "total_ms": round(tot, 3),
        "frames_per_s": round(1000.0 * B / tot, 1), "components_removed": 3, "data": note}
    log(f"doppler pipeline: {B} frames: prepare {part[0]:.2f} + forward {part[1]:.2f} + clutter "
        f"{part[2]:.2f} = {tot:.2f} ms")
    pf.close()
    del ye, ws, xe, wsc
    torch.cuda.empty_cache()

    # The clutter filter alone on a synthetic ensemble with a vessel (rank-3
    # tissue clutter 40 dB above blood, noise), 256 frames x 128^3.
    xe, _ = synth.doppler_ensemble_device((128, 128, 128), T=B, seed=11, device=dev)
    wsc = torch.empty(das.das_clutter_workspace_bytes(B), dtype=torch.uint8, device=dev)
    svc = torch.empty(B, device=dev)
    pwc = torch.empty(xe.shape[1], device=dev)
    das.das_clutter_filter(xe, 3, B, svc, pwc, None, wsc)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        das.das_clutter_filter(xe, 3, B, svc, pwc, None, wsc)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    forms["clutter_filter_power_doppler"] = {
        "ms_per_ensemble": round(ms, 3), "frames": B, "voxels": int(xe.shape[1]),
        "frames_per_s": round(1000.0 * B / ms, 1), "components_removed": 3,
        "data": "synthetic ensemble: rank-3 tissue clutter 40 dB above blood in a vessel, noise"}
    log(f"clutter filter + power Doppler: {B} frames x 128^3 in {ms:.2f} ms")
    del xe, wsc


if __name__ == "__main__":
    main()

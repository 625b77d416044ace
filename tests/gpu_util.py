"""Helpers for the GPU parity tests (imported by tests only)."""
import functools
import sys

import numpy as np
import torch

import oracle
import synth

# Parity bars (the FP32 and FP16 bars are the targets stated for the method;
# the others follow from the storage formats as explained beside each):
REL_L2_F32 = 1e-5      # FP32 storage and arithmetic vs the FP64 oracle
REL_L2_LOWP = 1e-3     # FP16 storage (FP32 arithmetic) vs the FP64 oracle
ABS_F32 = 1e-5         # elementwise |x - x_o| / max|x_o|, FP32
ABS_LOWP = 2e-3        # elementwise |x - x_o| / max|x_o|, FP16
# BF16 keeps 8 significant bits: round-to-nearest-even leaves a relative error
# of at most 2^-8 per sample, rms about 2^-7/sqrt(12) = 1.1e-3 to 1.7e-3 for
# Gaussian data, and the output error is of the same relative size.  Its bar
# is storage-limited: 4e-3 rel-L2, 6e-3 elementwise.
REL_L2_BF16 = 4e-3
ABS_BF16 = 6e-3
# FP8 (E4M3) keeps 4 significant bits, 2^4 times coarser than BF16: its
# rounding error and with it the bar are 16 times those of BF16 (measured with
# the oracle on Gaussian channel data: 2.6e-2 rel-L2).
REL_L2_FP8 = 16 * REL_L2_BF16
ABS_FP8 = 16 * ABS_BF16


def lowp_bars(storage):
    """(rel-L2, elementwise) bars against the oracle on the raw FP32 data."""
    if storage == "bf16":
        return REL_L2_BF16, ABS_BF16
    if storage == "fp8":
        return REL_L2_FP8, ABS_FP8
    return REL_L2_LOWP, ABS_LOWP


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(x, xo):
    x = np.asarray(x, np.float64)
    xo = np.asarray(xo, np.float64)
    return float(np.linalg.norm(x - xo) / np.linalg.norm(xo))


def check_close(x, xo, rel, absf, what=""):
    r = rel_l2(x, xo)
    a = float(np.max(np.abs(np.asarray(x, np.float64) - xo)) / np.max(np.abs(xo)))
    say(f"  {what}: rel-L2 {r:.3e} (bar {rel:g}), max|err|/max|x| {a:.3e} (bar {absf:g})")
    assert r <= rel, f"{what}: rel-L2 {r:.3e} > {rel:g}"
    assert a <= absf, f"{what}: max abs err {a:.3e} > {absf:g}"
    return r


def round_like_storage(y: np.ndarray, storage: str) -> np.ndarray:
    """The values a workspace of this storage type holds (round to nearest
    even; FP8 with one power-of-two scale per item of y[B, ...])."""
    if storage == "fp8":
        from oracle.storage import round_fp8_items
        return round_fp8_items(y)
    t = torch.from_numpy(np.asarray(y, np.float32))
    if storage == "f16":
        return t.to(torch.float16).to(torch.float64).numpy()
    if storage == "bf16":
        return t.to(torch.bfloat16).to(torch.float64).numpy()
    return t.to(torch.float64).numpy()


@functools.lru_cache(maxsize=4)
def cfg2_channel_data(device="cuda:0"):
    """cfg2 channel data simulated on the GPU with torch (float32 [Q, M, K])."""
    g, s, y = synth.cfg2_data(device=device)
    return g, y


def sample_voxels(g, count, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(g.N, size=min(count, g.N), replace=False))

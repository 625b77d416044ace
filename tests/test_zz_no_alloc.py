"""The allocation-free clutter filter entry point (static device workspace)
against das_clutter_filter with a caller workspace, on two calls in a row,
the second with a smaller ensemble (the static buffer keeps the first call's
contents).  Bars as in test_gpu_clutter: singular values squared within
2e-5 sigma_1^2, power image rel-L2 1e-4, filtered series 1e-3 (the Gram
matrix merges FP32 chunk sums with FP64 atomics in no fixed order, so the
two calls may differ at FP32 rounding level)."""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _das():
    from paper_2606_13259_amd import das
    return das


def _run_both(x, k_lo, k_hi, gpu):
    das = _das()
    T = x.shape[0]
    out = []
    for noalloc in (False, True):
        sv = torch.full((T,), float("nan"), device=gpu)
        pw = torch.full(x.shape[1:], float("nan"), device=gpu)
        xf = torch.full_like(x, float("nan"))
        if noalloc:
            das.das_clutter_filter_noalloc(x, k_lo, k_hi, sv, pw, xf)
        else:
            ws = torch.empty(das.das_clutter_workspace_bytes(T), dtype=torch.uint8, device=gpu)
            das.das_clutter_filter(x, k_lo, k_hi, sv, pw, xf, ws)
        torch.cuda.synchronize()
        out.append([t.cpu().numpy().astype(np.float64).reshape(T if t is sv else -1) if t is not xf
                    else t.cpu().numpy().astype(np.float64).reshape(T, -1) for t in (sv, pw, xf)])
    return out


def _compare(ref, got, what):
    (s0, p0, x0), (s1, p1, x1) = ref, got
    assert np.all(np.isfinite(s1)) and np.all(np.isfinite(p1)) and np.all(np.isfinite(x1))
    e_sig = float(np.max(np.abs(s1 ** 2 - s0 ** 2)) / s0[0] ** 2)
    e_pw = float(np.linalg.norm(p1 - p0) / np.linalg.norm(p0))
    e_xf = float(np.linalg.norm(x1 - x0) / np.linalg.norm(x0))
    say(f"  {what}: sigma^2 {e_sig:.2e}, power {e_pw:.2e}, filtered {e_xf:.2e}")
    assert e_sig <= 2e-5 and e_pw <= 1e-4 and e_xf <= 1e-3


def test_noalloc_matches_workspace_entry_point(gpu):
    # first call: 256 frames (the static buffer's limit), then a smaller ensemble
    for shape, T, k_lo, k_hi, seed in (((40, 32, 24), 256, 3, 256, 21), ((17, 13, 9), 48, 2, 40, 22)):
        x, _ = synth.doppler_ensemble(shape, T=T, seed=seed)
        xg = torch.from_numpy(np.ascontiguousarray(x)).to(gpu)
        say(f"no-alloc clutter filter: T={T}, N={xg.shape[1]}, keep {k_lo}..{k_hi - 1}")
        ref, got = _run_both(xg, k_lo, k_hi, gpu)
        _compare(ref, got, f"T={T}")


def test_noalloc_rejects_more_frames_than_its_buffer(gpu):
    das = _das()
    x = torch.zeros(257, 8, device=gpu)
    sv, pw = torch.empty(257, device=gpu), torch.empty(8, device=gpu)
    with pytest.raises(das.DasError) as e:
        das.das_clutter_filter_noalloc(x, 3, 257, sv, pw, None)
    assert e.value.status == das.DAS_ERR_INVALID_ARG

"""Write tests/golden/autofocus_scan.json: the oracle's focus criterion

    L(c) = sum_n |x~_n(c)|^4 / sum_n |x~_n(c)|^2

(x~ the complex volume beamformed from analytic channel data at sound speed
c) over the cfg5 volume sampled four times finer in depth (64 x 64 x 253
voxels, lateral spacing lambda/2, axial lambda/8, same depth range), with the
cfg5 channel data simulated at 1500 m/s, scanned over c in [1480, 1560] m/s:
coarse (2 m/s steps), then fine (0.5 m/s) around the coarse maximum.  Calls
only the oracle (FP64) and the seeded generators.

Run from the repository root: python tests/golden/make_autofocus_scan.py [workers]
"""
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import envelope as oenv  # noqa: E402


def main(workers):
    g, s, y = synth.cfg5_data(device="cpu")
    gf = synth.cfg5_focus_grid(g)
    lanes = oenv.analytic_lanes(y.numpy())

    def L(c):
        x, _ = oracle.forward_slabs_parallel(lanes, gf.replace(c=float(c)), workers=workers, chunk=8192)
        v = oenv.focus_criterion(x[0], x[1])
        print(f"  c = {c:7.2f} m/s  L = {v:.12e}", flush=True)
        return v

    coarse = np.arange(1480.0, 1560.0 + 1e-9, 2.0)
    lc = [L(c) for c in coarse]
    i = int(np.argmax(lc))
    c1 = float(coarse[i])
    fine = np.arange(max(1480.0, c1 - 2.0), min(1560.0, c1 + 2.0) + 1e-9, 0.5)
    lf = [L(c) for c in fine]
    c_best = float(fine[int(np.argmax(lf))])
    out = {"what": "oracle focus criterion sum|x~|^4 / sum|x~|^2 over the cfg5 volume sampled 4x finer "
                   "in depth (64 x 64 x 253 voxels) vs sound speed",
           "data": "synth.cfg5_data(device='cpu'): 50 targets (seed 6) + 2000 speckle (seed 60) at 1500 m/s",
           "grid": {"dims": list(gf.grid_dims), "spacing": list(gf.grid_spacing),
                    "origin": list(gf.grid_origin)},
           "coarse_c": coarse.tolist(), "coarse_L": lc, "fine_c": fine.tolist(), "fine_L": lf,
           "argmax_c": c_best, "interior": bool(0 < i < len(coarse) - 1)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autofocus_scan.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"argmax {c_best} m/s -> {path}")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1))

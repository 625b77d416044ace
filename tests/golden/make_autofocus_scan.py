"""Write tests/golden/autofocus_scan.json: the oracle's envelope energy
L(c) = sum_n |x~_n(c)|^2 over the full cfg5 volume (64^3 voxels, 16x16
array, 8 plane waves; channel data simulated at 1500 m/s on the CPU), scanned
over c in [1480, 1560] m/s, coarse (2 m/s) then fine (0.5 m/s) around the
coarse maximum, both within that range.  Calls only the oracle (FP64) and the seeded generators.

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
    lanes = oenv.analytic_lanes(y.numpy())

    def L(c):
        x, _ = oracle.forward_slabs_parallel(lanes, g.replace(c=float(c)), workers=workers, chunk=8192)
        v = float(np.sum(x ** 2))
        print(f"  c = {c:7.2f} m/s  L = {v:.10e}", flush=True)
        return v

    coarse = np.arange(1480.0, 1560.0 + 1e-9, 2.0)
    lc = [L(c) for c in coarse]
    c1 = float(coarse[int(np.argmax(lc))])
    fine = np.arange(max(1480.0, c1 - 2.0), min(1560.0, c1 + 2.0) + 1e-9, 0.5)
    lf = [L(c) for c in fine]
    c_best = float(fine[int(np.argmax(lf))])
    out = {"what": "oracle envelope energy over the full cfg5 volume vs sound speed",
           "data": "synth.cfg5_data(device='cpu'): 50 targets (seed 6) + 2000 speckle (seed 60) at 1500 m/s",
           "coarse_c": coarse.tolist(), "coarse_L": lc, "fine_c": fine.tolist(), "fine_L": lf,
           "argmax_c": c_best}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autofocus_scan.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"argmax {c_best} m/s -> {path}")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1))

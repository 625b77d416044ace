"""Writes nonzero_counts.json: the numbers of (voxel, element) pairs with a
nonzero receive weight for the benchmark workloads, counted by the FP64
oracle.  They are the unit counts of the algorithmic-work model (per pair,
per (pair, transmit) triple, per (triple, batch item)).

Run: python tests/golden/make_counts.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth   # noqa: E402

out = {}
for name, g in (("cfg1", synth.cfg1()), ("cfg2", synth.cfg2()), ("cfg5", synth.cfg5())):
    pnz, tnz = oracle.nonzero_counts(g)
    out[name] = {"N": g.N, "M": g.M, "Q": g.Q, "pairs_nonzero": pnz, "triples_nonzero": tnz,
                 "pairs_dense": g.N * g.M, "triples_dense": g.N * g.M * g.Q}
    print(name, out[name], flush=True)
with open(os.path.join(HERE, "nonzero_counts.json"), "w") as f:
    json.dump(out, f, indent=1)

"""The seeded input generators (CPU): the cfg4 motion ensemble follows the
random walk that ``synth.displaced`` defines."""
import numpy as np

import synth


def test_motion_walk_matches_displaced():
    g = synth.cfg2()
    s = synth.scatterers(g, 200, 10_000, seed_targets=3, seed_speckle=4)
    lam = synth.C_NOMINAL / synth.FC
    pos = synth.motion_positions(s, 9, synth.CFG4_SEED_BASE, lam)
    assert np.array_equal(pos[0], s.pos)
    for f in (1, 2, 8):
        assert np.array_equal(pos[f], synth.displaced(s, f, synth.CFG4_SEED_BASE, lam).pos)
    # per-frame steps: N(0, (lambda/40)^2) per axis, sub-wavelength
    steps = np.diff(np.stack(pos), axis=0)
    assert abs(steps.std() / (lam / 40) - 1) < 0.01
    assert np.abs(pos[8] - pos[0]).max() < lam

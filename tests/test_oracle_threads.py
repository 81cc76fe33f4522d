"""The timing-only pull form of the oracle (the CPU baseline on all cores)
computes the same sweeps as the sequential oracle: neutral fractions and
photon fields bit for bit (each receiver sums in the same order), tallies
to rounding."""
import math

import numpy as np

from paper_0912_4273_amd import gridgen as G
from oracle import Oracle


def test_threads_match_sequential():
    w = G.small_random(3000, seed=5, n_bins=42, box=3e21, rate=1e48, n_src=3, dt=3e13)
    sd = np.zeros((3, 3))
    sd[1] = [0.0, 0.0, 1.0]
    w = G.with_(w, src_dir=sd)
    a, b = Oracle(w), Oracle(w)
    a.run(9)
    b.run_threads(4, 4)
    b.run_threads(5, 3)      # the cached sender lists are reused
    sa, sb = a.state(), b.state()
    assert np.array_equal(sa["y"], sb["y"]) and np.array_equal(sa["photons"], sb["photons"])
    for key in ("emitted", "absorbed", "escaped", "in_flight"):
        assert math.isclose(sa["tallies"][key], sb["tallies"][key], rel_tol=1e-12), key
    # after a rotation the routing, and so the sender lists, change
    R = G.random_rotations(1, seed=3)[0]
    a.rotate(R)
    b.rotate(R)
    a.run(3)
    b.run_threads(3, 2)
    assert np.array_equal(a.state()["photons"], b.state()["photons"])

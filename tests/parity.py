"""Element-wise comparison helpers for GPU-vs-oracle parity tests."""
import numpy as np

# Tolerances per result (element passes if |gpu - ora| <= rtol*|ora| + atol).
# FP64 mode: same arithmetic as the oracle except the order of a few sums
# and the last ulp of exp/expm1 -> 1e-6 relative is loose by orders of
# magnitude.  FP32 transport: photons carry a 2^-24 relative rounding per
# hop; 1e-3 relative on x, y and the photon field.
TOL = {
    0: dict(xy=(1e-6, 1e-12), ph=(1e-6, 1e-12), tally=1e-9),
    1: dict(xy=(1e-3, 1e-6), ph=(1e-3, 1e-9), tally=1e-4),
}


def close(a, b, rtol, atol):
    a = np.asarray(a)
    b = np.asarray(b)
    bad = np.abs(a - b) > rtol * np.abs(b) + atol
    return (~bad).all(), int(bad.sum()), float(np.max(np.abs(a - b) / (np.abs(b) + atol)))


def assert_state_close(got, ref, precision, unit, what=""):
    t = TOL[precision]
    for key in ("x", "y"):
        ok, nbad, worst = close(got[key], ref[key], *t["xy"])
        assert ok, f"{what} {key}: {nbad} elements off, worst rel {worst:.3e}"
    if got.get("photons") is not None and ref.get("photons") is not None:
        rt, at = t["ph"]
        ok, nbad, worst = close(got["photons"], ref["photons"], rt, at * unit)
        assert ok, f"{what} photons: {nbad} elements off, worst rel {worst:.3e}"
    if got.get("nin") is not None and ref.get("nin") is not None:
        rt, at = t["ph"]
        ok, nbad, worst = close(got["nin"], ref["nin"], rt, at * unit)
        assert ok, f"{what} nin: {nbad} elements off, worst rel {worst:.3e}"
    for key in ("emitted", "absorbed", "escaped", "in_flight"):
        a, b = got["tallies"][key], ref["tallies"][key]
        scale = max(abs(ref["tallies"]["emitted"]), 1e-300)
        assert abs(a - b) <= t["tally"] * abs(b) + 1e-12 * scale, \
            f"{what} tally {key}: gpu {a!r} oracle {b!r}"
    assert got["tallies"]["sweeps"] == ref["tallies"]["sweeps"]


def assert_edges_close(got, ref, precision, unit, what=""):
    """Combined transport: every vertex holds the same layout on both sides,
    and the photons per edge slot agree within the photon tolerance."""
    lg = np.asarray(got["layout"]).astype(np.int64)
    lr = np.asarray(ref["layout"]).astype(np.int64)
    nbad = int(np.count_nonzero(lg != lr))
    assert nbad == 0, f"{what} layout: {nbad} vertices differ"
    rt, at = TOL[precision]["ph"]
    ok, nbad, worst = close(got["photons_e"], ref["photons_e"], rt, at * unit)
    assert ok, f"{what} photons_e: {nbad} elements off, worst rel {worst:.3e}"

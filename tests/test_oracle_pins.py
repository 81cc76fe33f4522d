"""The oracle against its pins (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

import analytic as A
import oracle_pins as P
from paper_0912_4273_amd import gridgen as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("pin", P.FAST_PINS, ids=[p.__name__ for p in P.FAST_PINS])
def test_fast_pin(pin):
    pin()


def test_stromgren_constants_match_paper():
    """The paper prints t_rec and r_S for Test 1 (Sect. 5.1); the analytic
    references reproduce them at the printed precision."""
    g = json.load(open(os.path.join(GOLDEN, "stromgren_test1.json")))
    p = g["parameters"]
    t_rec = A.recombination_time(p["n_H"], p["alpha_B"])
    r_s = A.stromgren_radius(p["rate"], p["n_H"], p["alpha_B"])
    pr = g["printed"]
    assert abs(t_rec - pr["t_rec_s"]) <= 0.005e15
    # the printed pair 3.86e15 s = 122.4 Myr implies 365-day years
    assert abs(t_rec / (365.0 * 86400.0 * 1e6) - pr["t_rec_myr"]) <= 0.05
    assert abs(r_s / G.KPC_CM - pr["r_s_kpc"]) <= 0.05
    # 500 Myr is about four recombination times, as the paper states
    assert abs(500.0 / (t_rec / G.MYR_S) - 4.0) < 0.1


def test_front_law_config1():
    worst = P.pin_front_law()
    assert worst < 0.08


@pytest.mark.parametrize("tau_switch", [1.0, 0.0])
def test_front_law_combined(tau_switch):
    """Combined transport with the paper's switch (optical depth 1) and pure
    ballistic transport (switch 0) both follow the front law of Test 1."""
    w = G.with_(G.config1(), transport=G.SX_TRANSPORT_COMBINED, tau_switch=tau_switch)
    worst = P.pin_front_law(w=w)
    assert worst < 0.08


def test_multihop_front_law():
    """Multi-hop steps let a 25 Myr step keep up with the front (Sect. 4.6)."""
    P.pin_multihop_front_law()


def test_diffuse_front_follows_case_b():
    P.pin_diffuse_front_follows_case_b()


def test_one_over_r2():
    P.pin_one_over_r2()


def test_front_velocity_consistent():
    """Eq. IFront_vel is the time derivative of Eq. IFront_pos."""
    r_s, t_rec = 5.4, 122.4
    t = np.linspace(5, 500, 50)
    h = 1e-4
    num = (A.front_radius(t + h, r_s, t_rec) - A.front_radius(t - h, r_s, t_rec)) / (2 * h)
    np.testing.assert_allclose(A.front_velocity(t, r_s, t_rec), num, rtol=1e-6)

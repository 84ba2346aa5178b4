"""Closed-form pins of the oracle's uniaxial test to failure.

Two grip particles joined by one or two springs: both ends are clamped, so
no dynamics enter and every record is known in closed form.  After n
increments of d_eps the right grip sits at L0 (1 + eps_n) (Section 3.1,
boundary particles displaced along x), a spring of rest length L0 has
length r_n = L0 (1 + eps_n), and its contribution to the virial stress
(Eq. 7: the spring vector times the force on the near end from the far
end, over the reference volume) is k r_n (r_n - L0) / Omega.  A spring
breaks for good at the first increment whose length exceeds
rc = L0 (1 + s) -- strict inequality, zero force from then on (Section
2.3 force routine; Section 4).

These cases fix the three derived quantities independently of the
oracle's code:
  * the stop rule: the first increment *after* the peak whose sigma_xx is
    *strictly* below drop x peak (drop = 0 never stops on a zero stress);
  * the strength: the peak sigma_xx;
  * the modulus window: increments that *ended* with no broken spring (at
    least the first one), least-squares slope through the origin.
"""
import math

import numpy as np
import pytest

from oracle import Net

L0 = 10.0
OMEGA = 7.0


def grip_pair(springs):
    """Two clamped grips at x = 0 and x = L0 joined by `springs`, each a
    (k, s) pair (rest length L0, critical length L0 (1 + s))."""
    X0 = np.array([[0.0, 0.0], [L0, 0.0]])
    m = len(springs)
    net = Net.network(2, X0, mass=[1.0, 1.0], c=[0.0, L0], grip=[1, 2],
                      sp=[0] * m, sq=[1] * m, k=[k for k, _ in springs],
                      r0=[L0] * m, rc=[L0 * (1.0 + s) for _, s in springs], omega=OMEGA)
    net.set_dynamics(0.01, 0.1, 0)
    return net


def strains(d_eps, n):
    # the applied strain is the running sum of the increments
    out, e = [], 0.0
    for _ in range(n):
        e += d_eps
        out.append(e)
    return np.array(out)


def closed_sigma(springs, eps):
    """sigma_xx after each increment: intact springs only."""
    sig = np.zeros(len(eps))
    for n, e in enumerate(eps):
        r = L0 * (1.0 + e)
        # a spring is intact at increment n if it never exceeded rc up to n
        k_on = sum(k for k, s in springs if not any(L0 * (1.0 + ee) > L0 * (1.0 + s)
                                                      for ee in eps[:n + 1]))
        sig[n] = k_on * r * (r - L0) / OMEGA
    return sig


def slope_through_origin(e, s):
    return float((e * s).sum() / (e * e).sum())


def test_single_spring_breaks_then_specimen_fails_one_increment_later():
    # s = 0.0225, d_eps = 0.005: intact at eps = 0.005 .. 0.02, broken at 0.025
    springs = [(0.8, 0.0225)]
    net = grip_pair(springs)
    res = net.run_to_failure(0.005, 3, 20, drop=0.01)
    eps = strains(0.005, 5)
    sig = closed_sigma(springs, eps)
    assert sig[4] == 0.0 and np.all(sig[:4] > 0)
    assert res["status"] == 0
    # stops at the first increment after the peak (inc 4) below 1 % of it,
    # i.e. increment 5 -- not at the peak itself, not later
    assert res["n_inc"] == 5
    assert np.allclose(res["sigma_xx"], sig, rtol=1e-12, atol=0)
    assert np.array_equal(res["n_broken"], [0, 0, 0, 0, 1])
    assert res["strength"] == pytest.approx(sig[3], rel=1e-12)
    # the modulus uses increments 1..4 (those that ended unbroken), not 5
    assert res["modulus"] == pytest.approx(slope_through_origin(eps[:4], sig[:4]), rel=1e-12)
    assert res["modulus"] != pytest.approx(slope_through_origin(eps, sig), rel=1e-6)
    ev = net.events()
    assert len(ev) == 1 and ev[0]["inc"] == 5 and ev[0]["step"] == 0 and ev[0]["id"] == 0
    r5 = L0 * (1.0 + eps[4])
    rc = L0 * 1.0225
    assert ev[0]["margin"] == pytest.approx((r5 - rc) / rc, rel=1e-9)


def test_drop_zero_never_stops_on_zero_stress():
    # with drop = 0 the rule "sigma_xx strictly below 0 x peak" never holds
    # for the zero stress of a broken specimen: it runs to the cap
    springs = [(0.8, 0.0225)]
    net = grip_pair(springs)
    res = net.run_to_failure(0.005, 3, 12, drop=0.0)
    assert res["n_inc"] == 12
    assert np.all(res["sigma_xx"][4:] == 0.0)
    assert res["strength"] == pytest.approx(closed_sigma(springs, strains(0.005, 4))[3], rel=1e-12)


def test_first_break_before_the_peak_limits_the_modulus_window():
    # a weak spring (k 0.2, s 0.0125) breaks at increment 3 while the stiff
    # one (k 1, s 0.0325) keeps the stress rising; the peak is at increment
    # 6, the stiff spring breaks at 7 and the test stops there
    springs = [(0.2, 0.0125), (1.0, 0.0325)]
    net = grip_pair(springs)
    res = net.run_to_failure(0.005, 3, 30, drop=0.01)
    eps = strains(0.005, 7)
    sig = closed_sigma(springs, eps)
    assert sig[2] > sig[1], "the first break must come before the peak"
    assert int(np.argmax(sig)) == 5 and sig[6] == 0.0
    assert res["n_inc"] == 7
    assert np.allclose(res["sigma_xx"], sig, rtol=1e-12, atol=0)
    assert np.array_equal(res["n_broken"], [0, 0, 1, 1, 1, 1, 2])
    assert res["strength"] == pytest.approx(sig[5], rel=1e-12)
    # window = increments 1 and 2 only; the increment with the first break
    # (3) and everything up to the peak are excluded
    assert res["modulus"] == pytest.approx(slope_through_origin(eps[:2], sig[:2]), rel=1e-12)
    for wrong in (3, 6):
        assert res["modulus"] != pytest.approx(slope_through_origin(eps[:wrong], sig[:wrong]),
                                               rel=1e-6)
    # closed-form modulus of the window: both springs at small strain give
    # (k1 + k2) L0^2 (1 + eps) / Omega per unit strain
    e2 = eps[:2]
    expect = float(((e2 * (1.2 * L0 * L0 * (1 + e2) * e2 / OMEGA)).sum()) / (e2 * e2).sum())
    assert res["modulus"] == pytest.approx(expect, rel=1e-12)
    ev = net.events()
    assert [(int(e["inc"]), int(e["id"])) for e in ev] == [(3, 0), (7, 1)]


def test_break_in_the_first_increment_keeps_a_one_increment_window():
    # broken at once: the window still holds the first increment (stress 0),
    # so the modulus is 0, and a zero peak never triggers the drop rule
    springs = [(1.0, 0.001)]
    net = grip_pair(springs)
    res = net.run_to_failure(0.005, 3, 6, drop=0.01)
    assert res["n_inc"] == 6
    assert np.all(res["sigma_xx"] == 0.0)
    assert res["modulus"] == 0.0 and res["strength"] == 0.0
    assert np.array_equal(res["n_broken"], [1] * 6)


def test_exact_threshold_does_not_break():
    # strict r > rc: a grip placed exactly at rc leaves the spring intact
    # (d_eps = 0.25 and s = 0.5 are exact in binary, so r_2 = rc exactly)
    springs = [(1.0, 0.5)]
    net = grip_pair(springs)
    res = net.run_to_failure(0.25, 2, 3, drop=0.01)
    eps = strains(0.25, 3)
    assert L0 * (1.0 + eps[1]) == L0 * 1.5
    assert np.array_equal(res["n_broken"], [0, 0, 1])
    assert res["sigma_xx"][1] == pytest.approx(1.0 * 15.0 * 5.0 / OMEGA, rel=1e-15)
    assert math.isclose(res["strength"], 75.0 / OMEGA, rel_tol=1e-15)

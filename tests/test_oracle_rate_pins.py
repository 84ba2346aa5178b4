"""Pins of the oracle's constant strain-rate protocol (the paper's loading:
Section 3.1 moves the boundary particles apart at a fixed strain rate, and
Section 2.3 applies that boundary displacement first in every time step).

* grip positions are exact functions of time: X0_x + (eps0 + s rate dt) c
  after s steps, and rate 0 stops them;
* a free particle between two grips on a line (two colinear springs, so the
  force is exactly linear in the positions) follows the two-step leapfrog
  form of velocity Verlet with damping,
      v_{n+1/2} = v_{n-1/2} (1 - gamma dt / m) + dt F_n / m,
      x_{n+1}   = x_n + dt v_{n+1/2},
  where F_n is evaluated with the grips already at the strain of step n
  (grips first); moving the grips after the force evaluation, or damping
  with the full-step velocity, changes the trajectory at first order.
"""
import numpy as np
import pytest

from oracle import Net

L0 = 10.0


def chain(k=0.5, m=2.0):
    # left grip at 0 (c = 0), free particle at L0, right grip at 2 L0 (c = 2 L0)
    X0 = np.array([[0.0, 0.0], [L0, 0.0], [2 * L0, 0.0]])
    net = Net.network(2, X0, mass=[1.0, m, 1.0], c=[0.0, L0, 2 * L0], grip=[1, 0, 2],
                      sp=[0, 1], sq=[1, 2], k=[k, k], r0=[L0, L0], rc=[1e9, 1e9], omega=1.0)
    return net


def test_grip_positions_follow_the_rate_exactly():
    net = chain()
    dt, rate = 0.05, 3e-4
    net.set_dynamics(dt, 0.2, 1)
    net.set_strain_rate(rate)
    for s in (1, 7, 40):
        net.relax(s if s == 1 else s - (1 if s == 7 else 7))
        x = net.x
        eps = 0.0 + s * (rate * dt)
        assert x[2, 0] == 2 * L0 + eps * (2 * L0)
        assert x[0, 0] == 0.0 and x[0, 1] == 0.0 and x[2, 1] == 0.0
        assert net.record()["eps"] == eps
    # rate 0: the grips stay where they are
    net.set_strain_rate(0.0)
    before = net.x[2, 0]
    net.relax(5)
    assert net.x[2, 0] == before


@pytest.mark.parametrize("gamma", [0.0, 0.3])
def test_free_particle_follows_the_leapfrog_recurrence(gamma):
    k, m, dt, rate = 0.5, 2.0, 0.05, 2e-3
    net = chain(k, m)
    net.set_dynamics(dt, gamma, 1)
    net.set_strain_rate(rate)
    n = 400
    xs = []
    for _ in range(n):
        net.relax(1)
        xs.append(net.x[1, 0])
    # two-step leapfrog from rest: v_{1/2} = 0 (no force at rest), x_0 = L0
    x, vh = L0, 0.0
    ref = []
    for s in range(1, n + 1):
        x = x + dt * vh                       # position update of step s
        xr = 2 * L0 + (s * (rate * dt)) * (2 * L0)  # grip placed first in step s
        F = k * (xr - x - L0) - k * (x - 0.0 - L0)
        vh = vh * (1.0 - gamma * dt / m) + dt * F / m
        ref.append(x)
    assert np.allclose(xs, ref, rtol=1e-13, atol=1e-12)
    # and the particle does move (the check is not vacuous)
    assert abs(xs[-1] - L0) > 1e-3


def test_rate_protocol_restarts_at_an_increment():
    # an increment resets the protocol's origin to the new strain
    net = chain()
    dt, rate = 0.05, 1e-3
    net.set_dynamics(dt, 0.2, 1)
    net.set_strain_rate(rate)
    net.relax(10)
    e10 = 10 * (rate * dt)
    net.apply_increment(0.01)
    assert net.record()["eps"] == e10 + 0.01
    net.relax(3)
    assert net.x[2, 0] == 2 * L0 + ((e10 + 0.01) + 3 * (rate * dt)) * (2 * L0)

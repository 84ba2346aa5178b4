"""Pins of the oracle's spring laws beyond the linear spring of Eq. 1-2
(the extensions the paper's closing section names): recoverable stiffness
of broken springs under compression and cubic (non-linear) elasticity.
Pinned by closed forms of a single spring, the force as the negative
gradient of the energy (central finite differences) on a perturbed
lattice, and energy conservation of the undamped integrator."""
import numpy as np
import pytest

from oracle import Net, Params
from paper_2201_04565_amd import inputs


def pair(r, k=2.0, r0=1.5, rc=10.0, law=0, c=0.0, broken=False, theta=0.3):
    u = np.array([np.cos(theta), np.sin(theta)])
    X0 = np.array([[0.0, 0.0], r0 * u])
    net = Net.network(2, X0, [1.0, 1.0], [0.0, 0.0], [0, 0], [0], [1], [k], [r0], [rc])
    net.set_spring_law(law, c)
    net.x = np.array([[0.0, 0.0], r * u])
    if broken:
        net.set_broken([1])
    return net, u


@pytest.mark.parametrize("r", [1.1, 1.4, 1.6, 2.3])
def test_cubic_single_spring_closed_form(r):
    k, r0, c = 2.0, 1.5, 3.0
    net, u = pair(r, k, r0, law=2, c=c)
    d = r - r0
    f = net.forces()
    want = k * d * (1.0 + c * d * d / (r0 * r0))
    assert np.allclose(f[0], want * u, rtol=1e-13, atol=1e-15)
    assert np.allclose(f[1], -want * u, rtol=1e-13, atol=1e-15)
    assert net.potential_energy() == pytest.approx(0.5 * k * d * d + 0.25 * k * c * d ** 4 / r0 ** 2, rel=1e-13)


@pytest.mark.parametrize("r,acts", [(1.2, True), (1.49, True), (1.51, False), (2.5, False)])
def test_recoverable_broken_spring(r, acts):
    k, r0 = 2.0, 1.5
    net, u = pair(r, k, r0, law=1, broken=True)
    f = net.forces()
    want = k * (r - r0) if acts else 0.0
    assert np.allclose(f[0], want * u, rtol=1e-13, atol=1e-15)
    assert net.potential_energy() == pytest.approx(0.5 * k * (r - r0) ** 2 if acts else 0.0, abs=1e-15)
    # under the linear law the broken spring carries nothing at any length
    net0, _ = pair(r, k, r0, law=0, broken=True)
    assert np.all(net0.forces() == 0.0)


def test_recoverable_intact_spring_is_linear():
    for r in (1.2, 1.8):
        a, _ = pair(r, law=1)
        b, _ = pair(r, law=0)
        assert np.array_equal(a.forces(), b.forces())


@pytest.mark.parametrize("law,c", [(1, 0.0), (2, 2.5), (2, -0.8)])
def test_force_is_minus_energy_gradient(law, c):
    img = inputs.bernoulli_two_phase(6, 5, 0.5, seed=9)
    net = Net.lattice(img, Params(k=[[0.4, np.nan], [np.nan, 1.0]], s=[[0.5, np.nan], [np.nan, 0.5]],
                                  mass=[1.0, 1.0]))
    net.set_spring_law(law, c)
    rng = np.random.default_rng(3)
    x = net.X0 + rng.uniform(-0.08, 0.08, size=(net.n, 2))
    net.x = x
    if law == 1:
        b = np.zeros(net.m, dtype=np.uint8)
        b[::3] = 1  # a third of the springs broken: the compressed ones act
        net.set_broken(b)
    F = net.forces()
    h = 1e-6
    G = np.zeros_like(x)
    for p in range(net.n):
        for e in range(2):
            xp, xm = x.copy(), x.copy()
            xp[p, e] += h
            xm[p, e] -= h
            net.x = xp
            up = net.potential_energy()
            net.x = xm
            G[p, e] = -(up - net.potential_energy()) / (2 * h)
    net.x = x
    assert np.max(np.abs(F - G)) <= 1e-7 * max(np.max(np.abs(F)), 1e-3)


def test_cubic_undamped_energy_is_conserved():
    # two free particles: velocity Verlet keeps the energy of the anharmonic
    # oscillator within O(dt^2) with no drift
    net, u = pair(2.1, k=1.0, r0=1.5, law=2, c=4.0)
    net.set_dynamics(0.01, 0.0)
    e = []
    for _ in range(200):
        net.relax(50)
        r = net.record()
        e.append(r["ke"] + r["pe"])
    e = np.array(e)
    assert np.max(np.abs(e - e[0])) <= 1e-3 * e[0]
    slope = np.polyfit(np.arange(len(e)), e, 1)[0]
    assert abs(slope) * len(e) <= 1e-5 * e[0]

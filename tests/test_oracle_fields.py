"""Pins of the oracle's local fields (oracle/fields.py) against what the
method and the mathematics fix, independent of the oracle's own code:

* the per-particle virial contributions add up to the bulk virial stress
  of Eq. 7 taken over the whole specimen (the record);
* a uniform triangular lattice under a small affine strain has, at every
  interior particle, the stress of the closed-form elastic constants
  C11 = 3 sqrt3 k / 4, C12 = C66 = sqrt3 k / 4; a simple-cubic face + edge
  lattice C11 = (k1 + 2 k2) / a, C12 = C44 = k2 / a;
* the least-squares map J of an affine deformation x = F X0 is F itself,
  so the Lagrangian strain is (F^T F - I) / 2 exactly, zero for a rigid
  rotation, at every particle whose nearest neighbours span the space;
* a broken spring contributes nothing to either end.
"""
import numpy as np
import pytest

from oracle import Net, Params
from oracle import fields as of
from paper_2201_04565_amd import inputs

SQ3 = np.sqrt(3.0)


def uniform(shape, k=1.0, kf=1.0, kd=1.0, a=1.0):
    img = np.zeros(shape, dtype=np.uint8)
    return Net.lattice(img, Params(k=[[k]], s=[[10.0]], mass=[1.0], a=a, k_face=kf, k_diag=kd,
                                   dt=0.01, gamma=0.0))


def interior(net, depth=2):
    X0 = net.X0
    lo, hi = X0.min(axis=0), X0.max(axis=0)
    ok = np.ones(net.n, dtype=bool)
    for c in range(net.dim):
        span = 1.0 if c == 0 or net.dim == 3 else SQ3 / 2
        ok &= (X0[:, c] > lo[c] + depth * span - 1e-9) & (X0[:, c] < hi[c] - depth * span + 1e-9)
    return ok


def test_particle_virials_sum_to_the_bulk_stress():
    wl = inputs.WORKLOADS["c1"]
    net = Net.lattice(inputs.c1_image(), Params(k=wl["k"], s=wl["s"], mass=wl["mass"], dt=wl["dt"],
                                               gamma=wl["gamma"]))
    for _ in range(8):
        net.apply_increment(0.01)
        net.relax(200)
    assert len(net.events()) > 0
    rec = net.record()
    s = of.particle_virial(net)
    total = s.sum(axis=0) / (net.n * of.site_volume(net, 1.0))
    assert np.max(np.abs(total - rec["sigma"][:2, :2])) <= 1e-12 * np.max(np.abs(rec["sigma"]))
    # radius-0 field averaged over all particles is the bulk stress too
    f0 = of.virial_stress_field(net, 1.0, 0)
    assert np.allclose(f0.mean(axis=0), rec["sigma"][:2, :2], rtol=1e-12, atol=0)


@pytest.mark.parametrize("eps", [np.array([[1e-6, 0.0], [0.0, 0.0]]),
                                 np.array([[3e-7, 2e-7], [2e-7, -5e-7]])])
def test_triangular_lattice_affine_stress(eps):
    k = 0.7
    net = uniform((14, 15), k=k)
    net.x = net.X0 @ (np.eye(2) + eps).T
    C11, C12, C66 = 3 * SQ3 * k / 4, SQ3 * k / 4, SQ3 * k / 4
    want = np.array([[C11 * eps[0, 0] + C12 * eps[1, 1], 2 * C66 * eps[0, 1]],
                     [2 * C66 * eps[0, 1], C12 * eps[0, 0] + C11 * eps[1, 1]]])
    for radius in (0, 1):
        f = of.virial_stress_field(net, 1.0, radius)[interior(net)]
        assert f.shape[0] > 50
        assert np.max(np.abs(f - want)) <= 1e-5 * np.max(np.abs(want))


def test_simple_cubic_affine_stress():
    k1, k2 = 1.0, 0.5
    net = uniform((7, 8, 9), kf=k1, kd=k2)
    e = 1e-6
    net.x = net.X0 @ np.diag([1 + e, 1.0, 1.0]).T
    C11, C12 = (k1 + 2 * k2), k2
    want = np.diag([C11 * e, C12 * e, C12 * e])
    f = of.virial_stress_field(net, 1.0, 0)[interior(net, 1)]
    assert f.shape[0] > 20
    assert np.max(np.abs(f - want)) <= 1e-5 * C11 * e


def rot2(t):
    return np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])


@pytest.mark.parametrize("F", [rot2(0.7), rot2(-1.1) @ np.array([[1.3, 0.2], [0.0, 0.8]]),
                               np.array([[1.05, 0.0], [0.0, 0.97]])])
def test_strain_of_affine_maps_2d(F):
    net = uniform((9, 11))
    net.x = net.X0 @ F.T + np.array([3.0, -2.0])
    eps = of.lagrangian_strain_field(net)
    want = 0.5 * (F.T @ F - np.eye(2))
    assert not np.isnan(eps).any()
    assert np.max(np.abs(eps - want)) <= 1e-12


def test_strain_of_affine_maps_3d():
    t = 0.4
    R = np.array([[1, 0, 0], [0, np.cos(t), -np.sin(t)], [0, np.sin(t), np.cos(t)]])
    F = R @ np.array([[1.1, 0.05, 0.0], [0.0, 0.9, 0.02], [0.0, 0.0, 1.02]])
    net = uniform((5, 6, 7))
    net.x = net.X0 @ F.T
    eps = of.lagrangian_strain_field(net)
    assert not np.isnan(eps).any()
    assert np.max(np.abs(eps - 0.5 * (F.T @ F - np.eye(3)))) <= 1e-12


def test_strain_undefined_without_spanning_neighbours():
    # a single row: every first-neighbour vector lies along x
    net = uniform((1, 6))
    eps = of.lagrangian_strain_field(net)
    assert np.isnan(eps).all()


def test_broken_spring_contributes_nothing():
    net = uniform((4, 5), k=2.0)
    rng = np.random.default_rng(0)
    net.x = net.X0 + rng.uniform(-0.02, 0.02, size=(net.n, 2))
    s_all = of.particle_virial(net)
    sp = net.springs()
    b = np.zeros(net.m, dtype=np.uint8)
    b[7] = 1
    net.set_broken(b)
    s_cut = of.particle_virial(net)
    p, q = int(sp["p"][7]), int(sp["q"][7])
    d = net.x[q] - net.x[p]
    r = np.linalg.norm(d)
    term = 0.5 * 2.0 * (r - sp["r0"][7]) / r * np.outer(d, d)
    assert np.allclose(s_all[p] - s_cut[p], term, atol=1e-15)
    assert np.allclose(s_all[q] - s_cut[q], term, atol=1e-15)
    others = np.ones(net.n, dtype=bool)
    others[[p, q]] = False
    assert np.array_equal(s_all[others], s_cut[others])

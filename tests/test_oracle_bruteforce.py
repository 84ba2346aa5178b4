"""Brute-force pins of the oracle on tiny lattices.

Independent re-derivations in numpy: neighbour pairs found by an all-pairs
distance search, forces as the finite-difference gradient of the potential,
break sets by exhaustive length checks, and the small-strain equilibrium as
a dense linear solve of the assembled stiffness matrix.
"""
import math

import numpy as np
import pytest

from oracle import Net, Params
from paper_2201_04565_amd import inputs

NAN = float("nan")


def two_phase(k_soft=0.1, k_stiff=1.0, s_soft=0.2, s_stiff=0.05, **kw):
    return Params(k=[[k_soft, NAN], [NAN, k_stiff]], s=[[s_soft, NAN], [NAN, s_stiff]],
                  mass=[1.0, 1.0], **kw)


def brute_pairs(X, rmax):
    D = np.linalg.norm(X[:, None, :] - X[None, :, :], axis=-1)
    i, j = np.nonzero((D < rmax) & (D > 0))
    return {(a, b) for a, b in zip(i, j) if a < b}, D


@pytest.mark.parametrize("shape", [(2, 2), (3, 4), (5, 6), (6, 5)])
def test_springs_are_all_nearest_pairs_2d(shape):
    img = inputs.bernoulli_two_phase(shape[1], shape[0], 0.5, seed=sum(shape))
    net = Net.lattice(img, two_phase())
    pairs, _ = brute_pairs(net.X0, 1.0 + 1e-9)
    sp = net.springs()
    assert set(zip(sp["p"].tolist(), sp["q"].tolist())) == pairs


@pytest.mark.parametrize("W", [2, 3, 4])
def test_springs_are_face_and_edge_pairs_3d(W):
    img = np.zeros((W, W, W), np.uint8)
    img.ravel()[np.random.default_rng(W).random(W ** 3) < 0.2] = 255
    net = Net.lattice(img, Params(k=[[1.0]], s=[[0.1]], mass=[1.0], void_value=255))
    pairs, D = brute_pairs(net.X0, math.sqrt(2.0) + 1e-9)
    sp = net.springs()
    assert set(zip(sp["p"].tolist(), sp["q"].tolist())) == pairs
    # rest lengths equal the reference distances
    assert np.allclose(sp["r0"], D[sp["p"], sp["q"]], atol=1e-14)


def _fd_check(net, x, h=1e-6):
    net.x = x
    F = net.forces()
    G = np.zeros_like(x)
    for p in range(net.n):
        for e in range(net.dim):
            xp = x.copy(); xp[p, e] += h
            xm = x.copy(); xm[p, e] -= h
            net.x = xp
            up = net.potential_energy()
            net.x = xm
            um = net.potential_energy()
            G[p, e] = -(up - um) / (2 * h)
    net.x = x
    return F, G


@pytest.mark.parametrize("img", [inputs.bernoulli_two_phase(4, 4, 0.5, seed=1),
                                 inputs.bernoulli_two_phase(5, 3, 0.5, seed=2)])
def test_forces_are_minus_gradient_2d(img):
    net = Net.lattice(img, two_phase(s_soft=10.0, s_stiff=10.0))
    x = net.X0 + inputs.perturbation(net.n, 2, 0.08, seed=11)
    F, G = _fd_check(net, x)
    assert np.allclose(F, G, atol=1e-8, rtol=1e-6)


def test_forces_are_minus_gradient_3d():
    img = np.zeros((3, 3, 3), np.uint8)
    img[1, 1, 1] = 1
    net = Net.lattice(img, Params(k=[[1.0, NAN], [NAN, 0.3]], s=[[10, NAN], [NAN, 10]],
                                  mass=[1.0, 1.0], k_face=1.0, k_diag=0.5))
    x = net.X0 + inputs.perturbation(net.n, 3, 0.08, seed=12)
    F, G = _fd_check(net, x)
    assert np.allclose(F, G, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_exhaustive_break_set(seed):
    img = inputs.bernoulli_two_phase(6, 6, 0.5, seed=seed)
    net = Net.lattice(img, two_phase(s_soft=0.08, s_stiff=0.03))
    x = net.X0 + inputs.perturbation(net.n, 2, 0.04, seed=100 + seed)
    net.x = x
    sp = net.springs()
    L = np.linalg.norm(x[sp["q"]] - x[sp["p"]], axis=1)
    expect = set(np.nonzero(L > sp["rc"])[0].tolist())
    assert 0 < len(expect) < net.m
    F = net.forces(commit=True)
    ev = net.events()
    assert set(ev["id"].tolist()) == expect
    assert np.allclose(ev["margin"], (L[ev["id"]] - sp["rc"][ev["id"]]) / sp["rc"][ev["id"]])
    # forces come from the surviving springs only
    keep = np.array([s not in expect for s in range(net.m)])
    d = x[sp["q"]] - x[sp["p"]]
    coef = np.where(keep, sp["k"] * (L - sp["r0"]) / L, 0.0)
    G = np.zeros_like(x)
    np.add.at(G, sp["p"], coef[:, None] * d)
    np.add.at(G, sp["q"], -coef[:, None] * d)
    assert np.allclose(F, G, atol=1e-15)


def _linear_equilibrium(net, eps):
    """Small-strain equilibrium K u = 0 with prescribed grip displacements."""
    X0 = net.X0
    sp = net.springs()
    mass, c, grip = net.particles()
    n, dim = net.n, net.dim
    K = np.zeros((n * dim, n * dim))
    for p, q, k in zip(sp["p"], sp["q"], sp["k"]):
        d = X0[q] - X0[p]
        nn = d / np.linalg.norm(d)
        B = k * np.outer(nn, nn)
        ip, iq = slice(p * dim, p * dim + dim), slice(q * dim, q * dim + dim)
        K[ip, ip] += B; K[iq, iq] += B; K[ip, iq] -= B; K[iq, ip] -= B
    u = np.zeros(n * dim)
    fixed = np.zeros(n * dim, bool)
    for p in np.nonzero(grip)[0]:
        fixed[p * dim:(p + 1) * dim] = True
        u[p * dim] = eps * c[p]
    free = ~fixed
    u[free] = np.linalg.solve(K[np.ix_(free, free)], -K[np.ix_(free, fixed)] @ u[fixed])
    return u.reshape(n, dim)


@pytest.mark.parametrize("W,H", [(6, 5), (8, 4)])
def test_quasistatic_limit_equals_linear_solve(W, H):
    img = inputs.bernoulli_two_phase(W, H, 0.5, seed=W * H)
    eps = 1e-6
    net = Net.lattice(img, two_phase(dt=0.05, gamma=1.0))
    u_lin = _linear_equilibrium(net, eps)
    net.apply_increment(eps)
    net.relax(40000)
    u = net.x - net.X0
    assert np.max(np.abs(u - u_lin)) < 1e-4 * np.max(np.abs(u_lin))
    assert net.record()["ke"] < 1e-24

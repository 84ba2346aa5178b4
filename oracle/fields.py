"""Local stress and strain fields of a particle-spring network (FP64 numpy).

TEST INFRASTRUCTURE ONLY: used by the test suite to check the library's
field kernels; the product package never imports it.  Every function is
pinned by tests/test_oracle_fields.py (a sum rule against the bulk stress,
the closed-form stress of a uniform lattice under affine strain, and the
exact strain of affine maps including rotations).

Definitions (Section 3.1, the virial stress and Lagrangian strain of the
field figure):

* virial contribution of particle k: s^k_ab = 1/2 sum_l (x^l_a - x^k_a)
  f^{kl}_b - m^k v^k_a v^k_b over the intact springs (k, l), f^{kl} the
  Eq. 2 force on k from l; tension is positive;
* virial stress over a domain of particles D: sigma = (1 / (|D| V_site))
  sum_{k in D} s^k (V_site: the area or volume of one lattice site); the
  fields use D = {p} (radius 0) or p and the particles it shares a spring
  with, broken or not (radius 1);
* Lagrangian strain: J is the least-squares affine map of p's first
  nearest-neighbour vectors (springs of the shortest rest length, broken
  or not) from the reference to the current configuration,
  J = (sum d d0^T)(sum d0 d0^T)^-1, and eps = (J^T J - I) / 2 (the
  Green-Lagrange reading of the garbled index form); NaN where the
  neighbour vectors do not span the space.
"""
from __future__ import annotations

import numpy as np


def _net_arrays(net):
    sp = net.springs()
    x = net.x
    v = net.v
    mass, _, _ = net.particles()
    return sp, x, v, mass


def particle_virial(net) -> np.ndarray:
    """s^k [n, dim, dim] (not divided by a volume)."""
    sp, x, v, mass = _net_arrays(net)
    n, dim = x.shape
    s = np.zeros((n, dim, dim))
    intact = sp["broken"] == 0
    p, q = sp["p"][intact], sp["q"][intact]
    d = x[q] - x[p]                                  # x^l - x^k for k = p
    r = np.sqrt(np.sum(d * d, axis=1))
    coef = sp["k"][intact] * (r - sp["r0"][intact]) / r
    f = coef[:, None] * d                            # force on p from q (Eq. 2)
    term = 0.5 * d[:, :, None] * f[:, None, :]       # (x^q - x^p)_a f^{pq}_b
    # the spring seen from q: (x^p - x^q)_a f^{qp}_b = (-d)_a (-f)_b, the same
    np.add.at(s, p, term)
    np.add.at(s, q, term)
    s -= mass[:, None, None] * v[:, :, None] * v[:, None, :]
    return s


def site_volume(net, a: float) -> float:
    return (np.sqrt(3.0) / 2.0) * a * a if net.dim == 2 else a ** 3


def neighbours(net):
    """Lists of the particles each particle shares a spring with."""
    sp = net.springs()
    nb = [[] for _ in range(net.n)]
    for p, q in zip(sp["p"], sp["q"]):
        nb[int(p)].append(int(q))
        nb[int(q)].append(int(p))
    return nb


def virial_stress_field(net, a: float, radius: int = 0) -> np.ndarray:
    """sigma^V per particle [n, dim, dim] over the radius-0 or radius-1 domain."""
    s = particle_virial(net)
    V = site_volume(net, a)
    if radius == 0:
        return s / V
    out = np.zeros_like(s)
    for p, nb in enumerate(neighbours(net)):
        dom = [p] + nb
        out[p] = s[dom].sum(axis=0) / (len(dom) * V)
    return out


def lagrangian_strain_field(net) -> np.ndarray:
    """eps^L per particle [n, dim, dim]; NaN where J is undefined."""
    sp = net.springs()
    x = net.x
    X0 = net.X0
    n, dim = x.shape
    r0min = np.min(sp["r0"]) if len(sp["r0"]) else 0.0
    first = np.abs(sp["r0"] - r0min) <= 1e-9 * max(r0min, 1.0)
    A = np.zeros((n, dim, dim))
    B = np.zeros((n, dim, dim))
    for p, q in zip(sp["p"][first], sp["q"][first]):
        d0 = X0[q] - X0[p]
        d = x[q] - x[p]
        for k, s0, s1 in ((p, d0, d), (q, -d0, -d)):
            A[k] += np.outer(s0, s0)
            B[k] += np.outer(s1, s0)
    eps = np.full((n, dim, dim), np.nan)
    eye = np.eye(dim)
    for k in range(n):
        if abs(np.linalg.det(A[k])) <= 1e-12 * max(np.abs(A[k]).max(), 1e-300) ** dim:
            continue
        J = B[k] @ np.linalg.inv(A[k])
        eps[k] = 0.5 * (J.T @ J - eye)
    return eps

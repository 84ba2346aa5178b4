"""GPU local fields (lsm_local_fields) against the oracle's (oracle/fields.py):
virial stress of Eq. 7 over radius-0 and radius-1 domains and the
Lagrangian strain (Section 3.1 field figure), element by element, on 2D
and 3D lattices fractured by a GPU run: the oracle's network is given the
GPU's positions, velocities and broken springs, so both evaluate the fields
of one configuration."""
import sys

import numpy as np
import pytest

from oracle import Net, Params
from oracle import fields as of
from paper_2201_04565_amd import inputs

pytestmark = pytest.mark.gpu

NAN = float("nan")


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lsm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_04565_amd import lsm as _lsm
    _lsm.load_library()
    return _lsm


CASES = [
    ("c1 32x32", lambda: inputs.c1_image(), "c1", 8, 300, 0.01),
    ("brick 90x37", lambda: inputs.brick_and_mortar(90, 37, seed=1), "c2", 4, 300, 0.006),
    ("grf 18^3", lambda: inputs.gaussian_random_field_3d(18, corr_len=3.0, seed=4), "c3", 3, 300, 0.012),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32k"])
@pytest.mark.parametrize("name,make,wlname,n_inc,steps,d_eps", CASES)
def test_local_fields_match_oracle(lsm, precision, name, make, wlname, n_inc, steps, d_eps):
    img = make()
    wl = inputs.WORKLOADS[wlname]
    say(f"local fields {name} {precision}: {n_inc} x relax({steps}), d_eps {d_eps}")
    o = Net.lattice(img, Params(k=wl["k"], s=wl["s"], mass=wl["mass"], a=wl.get("a", 1.0),
                                k_face=wl.get("k_face", 1.0), k_diag=wl.get("k_diag", 1.0), dt=wl["dt"],
                                gamma=wl["gamma"], void_value=wl.get("void_value", -1)))
    g = lsm.Lattice.from_workload(wl, img, precision=precision)
    for _ in range(n_inc):
        g.apply_increment(d_eps)
        g.relax(steps)
    ev_g = g.read_broken()
    assert len(ev_g) > 0, "the case should break springs"
    broken = np.zeros(o.m, dtype=np.uint8)
    broken[ev_g["id"]] = 1
    o.set_broken(broken)
    o.x = g.x
    o.v = g.v
    a = wl.get("a", 1.0)
    tol = 1e-10 if precision == "fp64" else 1e-8
    for radius in (0, 1):
        s_g, e_g = g.local_fields(radius)
        s_o = of.virial_stress_field(o, a, radius)
        scale = np.max(np.abs(s_o))
        err = np.max(np.abs(s_g - s_o)) / scale
        say(f"  radius {radius}: stress largest error {err:.2e} of max |sigma| {scale:.3e}")
        assert err <= tol
    e_o = of.lagrangian_strain_field(o)
    nan_o, nan_g = np.isnan(e_o), np.isnan(e_g)
    assert np.array_equal(nan_o, nan_g)
    ok = ~nan_o
    errs = np.max(np.abs(e_g[ok] - e_o[ok]))
    say(f"  strain: {int(nan_o.any(axis=(1, 2)).sum())} undefined, largest error {errs:.2e} "
        f"(max |eps| {np.max(np.abs(e_o[ok])):.3e})")
    assert errs <= tol * max(np.max(np.abs(e_o[ok])), 1e-3)


def test_local_fields_bad_arguments(lsm):
    import torch
    g = lsm.Lattice.from_workload(inputs.WORKLOADS["c1"], inputs.c1_image(), precision="fp64")
    buf = torch.zeros(g.n * 4, dtype=torch.float64, device="cuda:0")
    with pytest.raises(lsm.LsmError):
        g._check(g._L.lsm_local_fields(g._h, 2, lsm.C.c_void_p(buf.data_ptr()), lsm.C.c_void_p(buf.data_ptr())))
    g.apply_increment(0.01)
    with pytest.raises(lsm.LsmError):  # half-step velocities
        g.local_fields(0)
    g.relax(10)
    g.local_fields(1)

"""GPU spring laws beyond the linear spring (recoverable stiffness under
compression, cubic elasticity; the extensions of the paper's closing
section) against the oracle running the same law and protocol: broken-
spring sequence identical before the first near-tie, stress and energies
per increment within 1e-4 (FP64) or 1e-3 (FP32-compensated) up to it.  The
recoverable law is loaded in tension (cracks open) and then compressed back
past zero strain, so broken springs close and act; the run must differ
from the linear law's."""
import sys

import numpy as np
import pytest

from oracle import Net, Params
from paper_2201_04565_amd import inputs
from tests.parity import compare_events, compare_records

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-4, 1e-9), "fp32k": (1e-3, 1e-5)}


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


PROTOCOLS = {
    "cubic": [0.01] * 8,
    "recover": [0.015] * 5 + [-0.015] * 8,
    "linear": [0.015] * 5 + [-0.015] * 8,
}
LAW_ID = {"linear": 0, "recover": 1, "cubic": 2}


def run(lsm, img, wl, precision, law, c, steps):
    o = Net.lattice(img, Params(k=wl["k"], s=wl["s"], mass=wl["mass"], a=wl.get("a", 1.0),
                                k_face=wl.get("k_face", 1.0), k_diag=wl.get("k_diag", 1.0), dt=wl["dt"],
                                gamma=wl["gamma"], void_value=wl.get("void_value", -1)))
    o.set_spring_law(LAW_ID[law], c)
    g = lsm.Lattice.from_workload(wl, img, precision=precision, spring_law=law, law_c=c)
    # 2D lattices run the gather kernel under a non-linear law, single-phase
    # 3D ones the LDS-window compact kernel
    assert law == "linear" or g.launch()["variant"] == ("compact" if img.ndim == 3 else "gather")
    ro, rg = [], []
    for d_eps in PROTOCOLS[law]:
        for x in (o, g):
            x.apply_increment(d_eps)
            x.relax(steps)
        ro.append(o.record())
        rg.append(g.read_state())
    return o, g, ro, rg


CASES = [("c1 32x32", lambda: inputs.c1_image(), "c1", 300),
         ("grf 16^3", lambda: inputs.gaussian_random_field_3d(16, corr_len=3.0, seed=6), "c3", 200)]


@pytest.mark.parametrize("precision", ["fp64", "fp32k"])
@pytest.mark.parametrize("law,c", [("cubic", 5.0), ("recover", 0.0)])
@pytest.mark.parametrize("name,make,wlname,steps", CASES)
def test_spring_law_matches_oracle(lsm, name, make, wlname, steps, law, c, precision):
    img = make()
    wl = inputs.WORKLOADS[wlname]
    say(f"{law} law {name} {precision}: increments {PROTOCOLS[law]}")
    o, g, ro, rg = run(lsm, img, wl, precision, law, c, steps)
    rtol, tie = TOL[precision]
    ev_o, ev_g = o.events(), g.read_broken()
    assert len(ev_o) > 0
    div_inc, k = compare_events(ev_o, ev_g, tie)
    n = compare_records(ro, rg, rtol, img.ndim, upto_inc=div_inc)
    say(f"  {len(ev_o)} oracle events, {k} identical before the first near-tie; {n} records compared")
    # FP32 break decisions tie early in these fast-loaded 3D runs (a few
    # hundred breaks per increment); FP64 runs agree over the whole protocol
    assert k >= 1
    assert n >= (3 if precision == "fp64" else 1)
    if law == "recover" and precision == "fp64":
        # the same protocol under the linear law: once the cracks close, the
        # recovered springs carry compression and the stress differs
        _, _, ro_lin, _ = run(lsm, img, wl, precision, "linear", 0.0, steps)
        last = ro[-1]["sigma"][0, 0], ro_lin[-1]["sigma"][0, 0]
        say(f"  final sigma_xx: recoverable {last[0]:.6g}, linear {last[1]:.6g}")
        assert last[0] < last[1] and abs(last[0] - last[1]) > 1e-3 * abs(last[1])


@pytest.mark.parametrize("precision", ["fp64", "fp32k"])
@pytest.mark.parametrize("law,c", [("cubic", 5.0), ("recover", 0.0)])
def test_spring_law_compact_is_bitwise_the_gather_kernel(lsm, law, c, precision):
    # the interior steps of the LDS-window compact kernel under each law
    # against the gather kernel: a random field and a solid block whose
    # windows exceed the LDS pool (neighbours read from global memory), the
    # law's protocol with fracture (and, for the recoverable law, closing
    # cracks); state, break bits and events equal
    wl = inputs.WORKLOADS["c3"]
    cases = [("grf 18^3", inputs.gaussian_random_field_3d(18, corr_len=3.0, seed=4), 250),
             ("solid 330x4x4", np.zeros((4, 4, 330), np.uint8), 150)]
    for name, img, steps in cases:
        say(f"{law} law compact vs gather {name} {precision}")
        out = []
        for variant in ("gather", "compact"):
            g = lsm.Lattice.from_workload(wl, img, precision=precision, spring_law=law, law_c=c)
            g.set_launch(variant)
            assert g.launch()["variant"] == variant
            for d_eps in PROTOCOLS[law]:
                g.apply_increment(d_eps)
                g.relax(steps)
            out.append((g.save_state(), g.read_broken()))
        assert len(out[0][1]) > 0, "the case should break springs"
        say(f"  {len(out[0][1])} events")
        assert np.array_equal(out[1][1], out[0][1])
        assert out[1][0] == out[0][0]

"""GPU tests of the batched path: every specimen of a batch is bitwise the
single-lattice row-sweep run of the same image (same kernels, same per-site
order, same reduction order), and the derived modulus and strength follow
the oracle's run-to-failure."""
import sys

import numpy as np
import pytest

from oracle import Net, Params
from paper_2201_04565_amd import inputs
from tests.parity import compare_events

pytestmark = pytest.mark.gpu


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


def specimens():
    sizes = [24, 40, 64, 70, 33, 96]
    return [inputs.circular_inclusions(L, seed=1000 + i) for i, L in enumerate(sizes)]


@pytest.mark.parametrize("precision", ["fp64", "fp32k"])
def test_batch_equals_single_lattice_runs(lsm, precision):
    wl = inputs.WORKLOADS["c4"]
    imgs = specimens()
    say(f"batch of {len(imgs)} inclusion specimens {precision}, 0.5% x 300 steps to failure")
    b = lsm.Batch.from_workload(wl, imgs, precision=precision)
    # a loose failure threshold (25 % of the peak) so that specimens retire
    # at different increments within the test
    b.run(wl["d_eps"], 300, 40, drop=0.25)
    res = b.read()
    say(f"  increments per specimen: {res['n_inc'].tolist()}")
    assert np.all(res["n_inc"] >= 2)
    assert (res["n_inc"] < 40).any() and len(set(res["n_inc"].tolist())) > 1
    for s, img in enumerate(imgs):
        g = lsm.Lattice.from_workload(wl, img, precision=precision)
        # the batch runs the row sweeps (a small single lattice would
        # default to the one-workgroup kernel, whose arithmetic is the
        # gather kernel's)
        g.set_launch("sweep2" if precision == "fp32k" else "sweep")
        sx = []
        for _ in range(res["n_inc"][s]):
            g.apply_increment(wl["d_eps"])
            g.relax(300)
            sx.append(g.read_state()["sigma"][0, 0])
        k = res["n_inc"][s]
        assert np.array_equal(np.array(sx), res["sigma_xx"][s, :k]), f"specimen {s}"
        assert np.all(np.isnan(res["sigma_xx"][s, k:]))
        assert g.n_broken() == res["n_broken"][s]


def test_batch_rows_independent_and_order_free(lsm):
    wl = inputs.WORKLOADS["c4"]
    imgs = specimens()
    say("batch launch-shape independence and specimen order")
    out = []
    cases = ((4, None, "sweep"), (13, None, "sweep"), (4, [5, 3, 1, 0, 2, 4], "sweep"),
             (4, None, "sweep2"), (7, None, "sweep2"), (16, [5, 3, 1, 0, 2, 4], "sweep2"))
    for rows, order, variant in cases:
        use = imgs if order is None else [imgs[i] for i in order]
        b = lsm.Batch.from_workload(wl, use, precision="fp32k")
        b.set_launch(rows, 1, variant)
        assert b.launch()["steps_per_launch"] == (2 if variant == "sweep2" else 1)
        b.run(wl["d_eps"], 200, 25)
        r = b.read()
        if order is not None:
            inv = np.argsort(order)
            r = {k: v[inv] for k, v in r.items()}
        out.append(r)
    for r in out[1:]:
        for key in ("sigma_xx", "n_inc", "modulus", "strength", "n_broken"):
            assert np.array_equal(np.nan_to_num(r[key]), np.nan_to_num(out[0][key])), key


def test_batch_autotune_keeps_results(lsm):
    wl = inputs.WORKLOADS["c4"]
    imgs = specimens()
    say("batch autotune before the run leaves the results unchanged")
    out = []
    for tune in (False, True):
        b = lsm.Batch.from_workload(wl, imgs, precision="fp32k")
        if tune:
            res = b.autotune(20)
            assert len(res) >= 4 and all(r[3] > 0 for r in res)
            assert {r[0] for r in res} == {"sweep", "sweep2"}
            say(f"  picked {b.launch()} of {len(res)} candidates")
        b.run(wl["d_eps"], 200, 25)
        out.append(b.read())
    for key in ("sigma_xx", "n_inc", "modulus", "strength", "n_broken"):
        assert np.array_equal(np.nan_to_num(out[1][key]), np.nan_to_num(out[0][key])), key


def test_batch_derived_against_oracle(lsm):
    wl = inputs.WORKLOADS["c4"]
    imgs = specimens()[:4]
    say("batch fp64 modulus/strength/failure vs oracle run_to_failure")
    b = lsm.Batch.from_workload(wl, imgs, precision="fp64")
    b.run(wl["d_eps"], 300, 40)
    res = b.read()
    prm = Params(k=wl["k"], s=wl["s"], mass=wl["mass"], dt=wl["dt"], gamma=wl["gamma"])
    for s, img in enumerate(imgs):
        o = Net.lattice(img, prm)
        ro = o.run_to_failure(wl["d_eps"], 300, 40)
        # the modulus uses the increments before the first break, which come
        # before any fracture-path divergence
        assert res["modulus"][s] == pytest.approx(ro["modulus"], rel=1e-4)
        # curves agree until the first increment that ends with broken springs
        k = max(int(np.argmax(ro["n_broken"] > 0)), 1) if (ro["n_broken"] > 0).any() else ro["n_inc"]
        assert np.allclose(res["sigma_xx"][s, :k], ro["sigma_xx"][:k], rtol=1e-4)
        # strength within the paper's qualitative agreement band after fracture
        assert res["strength"][s] == pytest.approx(ro["strength"], rel=0.05)


def test_c4_stratified_sample_against_oracle(lsm):
    # the C4 workload (FP32 compensated, 0.5 % x 500 steps, failure rule,
    # cap 64) on one specimen per side length, against the FP64 oracle's
    # run to failure: the full protocol for sides 64-128, the first eight
    # increments for 192 and 256 (the oracle needs about a minute per
    # 256-side specimen for all 64)
    wl = inputs.WORKLOADS["c4"]
    for sides, cap in (((64, 96, 128), wl["max_inc"]), ((192, 256), 8)):
        imgs = [inputs.circular_inclusions(L, seed=1000 + i) for i, L in enumerate(sides)]
        say(f"c4 sample sides {sides} fp32k, {cap} increments x {wl['steps']} steps vs oracle")
        b = lsm.Batch.from_workload(wl, imgs, precision="fp32k")
        b.run(wl["d_eps"], wl["steps"], cap)
        res = b.read()
        prm = Params(k=wl["k"], s=wl["s"], mass=wl["mass"], dt=wl["dt"], gamma=wl["gamma"])
        for s, img in enumerate(imgs):
            ro = Net.lattice(img, prm).run_to_failure(wl["d_eps"], wl["steps"], cap)
            say(f"  side {img.shape[0]}: {ro['n_inc']} increments, modulus {ro['modulus']:.6g}")
            assert res["modulus"][s] == pytest.approx(ro["modulus"], rel=1e-3)
            k = max(int(np.argmax(ro["n_broken"] > 0)), 1) if (ro["n_broken"] > 0).any() else ro["n_inc"]
            peak = np.max(np.abs(ro["sigma_xx"][:ro["n_inc"]]))
            assert np.allclose(res["sigma_xx"][s, :k], ro["sigma_xx"][:k], rtol=1e-3, atol=1e-3 * peak)
            assert res["strength"][s] == pytest.approx(ro["strength"], rel=0.05)

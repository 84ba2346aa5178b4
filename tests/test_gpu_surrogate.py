"""What the trained surrogate gains over the model alone, and its fallback
(GPU).

64 x 64 inclusion specimens labelled by the batched model; a 3-member
ensemble trained on them must (a) predict the modulus far better than the
best input-free guess (the training mean), (b) keep the specimens it
accepts -- ensemble spread at or below a gate calibrated on a held-out
split -- within 5 % modulus error at the 95th percentile on a test split,
(c) answer accepted specimens orders of magnitude faster than the batched
model labels them (how many it accepts depends on how well it is trained:
this small ensemble about a third, the 128 x 128 one of the benchmark all),
and (d) send images unlike its training set (all soft,
a one-pixel checkerboard, inclusions of radius 16-28 px) back to the
model, whose answers are bitwise those of a direct batched run."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def trained():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_04565_amd import surrogate as S

    say("labels: 1536 train + 256 validation + 256 test 64x64 specimens, 64 increments x 500 steps")
    img_tr = S.specimen_images(1536, 10 ** 6, size=64)
    img_va = S.specimen_images(256, 3 * 10 ** 6, size=64)
    img_te = S.specimen_images(256, 2 * 10 ** 6, size=64)
    lab_tr, lab_va, lab_te = S.label(img_tr), S.label(img_va), S.label(img_te)
    say(f"  labelling {lab_tr.seconds + lab_va.seconds + lab_te.seconds:.1f} s")
    sur = S.Surrogate(k=3, size=64, batch=128, seed=1)
    sur.fit(img_tr, S.targets(lab_tr), epochs=24, lr=2e-3)
    say(f"  training {sur.train_seconds:.1f} s")
    return S, sur, (img_tr, lab_tr), (img_va, lab_va), (img_te, lab_te)


def test_surrogate_gain_small(trained):
    S, sur, (img_tr, lab_tr), (img_va, lab_va), (img_te, lab_te) = trained
    pred, spread, t_inf = sur.predict(img_te)
    err = np.abs(pred[:, -1] - lab_te.modulus) / lab_te.modulus
    base = np.abs(lab_tr.modulus.mean() - lab_te.modulus) / lab_te.modulus
    say(f"  modulus error: surrogate mean {err.mean():.4f}, training-mean guess {base.mean():.4f}")
    assert err.mean() < 0.5 * base.mean()
    cal = S.calibrate_gate(sur, img_va, lab_va, target_p95=0.04)
    say(f"  gate calibrated on validation: {cal}")
    res = S.evaluate(sur, img_te, lab_te, gate=cal["gate"])
    say(f"  gated: fallback {res['fallback_rate']:.3f}, accepted p95 {res['accepted_modulus_err_p95']:.4f}, "
        f"pipeline error mean {res['pipeline_modulus_err_mean']:.4f}, p95 {res['pipeline_modulus_err_p95']:.4f}")
    assert res["accepted_modulus_err_p95"] <= 0.05
    assert res["pipeline_modulus_err_p95"] <= 0.05
    per_spec_inf = t_inf / len(img_te)
    per_spec_lsm = lab_te.seconds / len(img_te)
    say(f"  per specimen: surrogate {per_spec_inf * 1e6:.1f} us, batched model {per_spec_lsm * 1e3:.2f} ms")
    assert per_spec_inf * 100 < per_spec_lsm


def test_out_of_distribution_images_fall_back(trained):
    from paper_2201_04565_amd import inputs
    S, sur, _, (img_va, lab_va), _ = trained
    cal = S.calibrate_gate(sur, img_va, lab_va, target_p95=0.04)
    ood = {"all soft": [inputs.uniform_phase(64, inputs.SOFT)],
           "checkerboard": [inputs.checkerboard(64)],
           "radius 16-28": [inputs.circular_inclusions(64, seed=4 * 10 ** 6 + i, r_min=16.0, r_max=28.0)
                            for i in range(4)]}
    imgs = np.stack([im for v in ood.values() for im in v])
    a = S.answer(sur, imgs, cal["gate"])
    k = 0
    for name, v in ood.items():
        say(f"  {name}: spread {np.round(a.spread[k:k + len(v)], 4).tolist()} (gate {cal['gate']:.4f}), "
            f"fallback {a.fallback[k:k + len(v)].tolist()}")
        assert a.fallback[k:k + len(v)].any(), f"{name} images were accepted"
        k += len(v)
    # the fallback answers are the batched model's, bit for bit: each
    # specimen run alone gives what the fallback batch gave it
    for r, i in enumerate(np.nonzero(a.fallback)[0]):
        one = S.label(imgs[i:i + 1])
        assert one.modulus[0] == a.modulus[i] and one.strength[0] == a.strength[i]
        assert np.array_equal(one.curves[0], a.curves[i])

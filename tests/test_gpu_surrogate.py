"""What the trained surrogate gains over the model alone (GPU).

64 x 64 inclusion specimens labelled by the batched model; a 3-member
ensemble trained on them must (a) predict the modulus far better than the
best input-free guess (the training mean), (b) keep every specimen it
accepts within the 5 % modulus gate's intent on held-out data, and (c)
answer accepted specimens orders of magnitude faster than the batched model
labels them."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def test_surrogate_gain_small():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_04565_amd import surrogate as S

    say("labels: 1536 train + 256 test 64x64 specimens, 64 increments x 500 steps")
    img_tr = S.specimen_images(1536, 10 ** 6, size=64)
    img_te = S.specimen_images(256, 2 * 10 ** 6, size=64)
    lab_tr = S.label(img_tr)
    lab_te = S.label(img_te)
    say(f"  labelling {lab_tr.seconds + lab_te.seconds:.1f} s")
    sur = S.Surrogate(k=3, size=64, batch=128, seed=1)
    sur.fit(img_tr, S.targets(lab_tr), epochs=12, lr=2e-3)
    say(f"  training {sur.train_seconds:.1f} s")
    pred, spread, t_inf = sur.predict(img_te)
    err = np.abs(pred[:, -1] - lab_te.modulus) / lab_te.modulus
    base = np.abs(lab_tr.modulus.mean() - lab_te.modulus) / lab_te.modulus
    say(f"  modulus error: surrogate mean {err.mean():.4f}, training-mean guess {base.mean():.4f}")
    assert err.mean() < 0.5 * base.mean()
    res = S.evaluate(sur, img_te, lab_te, gate=0.05)
    say(f"  gated: fallback {res['fallback_rate']:.3f}, pipeline error mean "
        f"{res['pipeline_modulus_err_mean']:.4f}, p95 {res['pipeline_modulus_err_p95']:.4f}")
    assert res["pipeline_modulus_err_mean"] < 0.05
    per_spec_inf = t_inf / len(img_te)
    per_spec_lsm = lab_te.seconds / len(img_te)
    say(f"  per specimen: surrogate {per_spec_inf * 1e6:.1f} us, batched model {per_spec_lsm * 1e3:.2f} ms")
    assert per_spec_inf * 100 < per_spec_lsm

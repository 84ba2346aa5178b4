"""The allocation-free loss entry point (GPU): lsm_cnn_mse_noalloc against
lsm_cnn_mse, bit for bit, on two calls in a row -- the second after a
forward pass over a smaller batch -- through the C ABI."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def test_mse_noalloc_matches_mse():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_04565_amd import cnn, inputs
    from paper_2201_04565_amd.surrogate import _he_normal

    net = cnn.Network(size=32, batch=16, outputs=65)
    net.set_params(_he_normal(net, 3))
    rng = np.random.default_rng(5)
    for B in (16, 5):
        say(f"mse vs mse_noalloc, batch {B}")
        imgs = np.stack([inputs.circular_inclusions(32, seed=700 + i) for i in range(B)])
        x = torch.from_numpy(imgs).to("cuda:0")
        tgt = torch.from_numpy(rng.normal(size=(B, 65)).astype(np.float32)).to("cuda:0")
        net.forward(x)
        loss_ref = net.mse(tgt).clone()
        dy_ref = torch.from_numpy(net.buffer("dout")[: B * 65].reshape(B, 65)).to("cuda:0")
        dy = torch.full((B, 65), float("nan"), dtype=torch.float32, device="cuda:0")
        loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda:0")
        net.mse_noalloc(tgt, dy, loss)
        torch.cuda.synchronize()
        assert torch.equal(dy, dy_ref)
        assert torch.equal(loss.reshape(-1)[:1], loss_ref.reshape(-1)[:1])
        say(f"  loss {float(loss[0]):.6f}, {dy.numel()} gradient values equal")

"""GPU parity of the surrogate network against the FP64 oracle.

The oracle runs in its BF16-emulation mode (weights and stored activations
rounded to bfloat16 where the GPU stores them), so the remaining difference
is FP32 vs FP64 accumulation plus the rare activation that rounds to the
other side of a bfloat16 boundary."""
import sys

import numpy as np
import pytest

from oracle import cnn_oracle as co

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cnn():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_04565_amd import cnn
    return torch, cnn


def bf16_tensor(torch, a):
    return torch.from_numpy(co.bf16_round(a).astype(np.float32)).to("cuda:0").to(torch.bfloat16)


@pytest.mark.parametrize("layer,cin,cout,H", [(1, 32, 64, 16), (2, 64, 128, 16), (4, 128, 256, 16)])
def test_conv_mfma_layer(torch_cnn, layer, cin, cout, H):
    torch, cnn = torch_cnn
    size = H * (2 ** layer)
    say(f"conv layer {layer}: {cin}->{cout} at {H}x{H}")
    net = cnn.Network(size=size, batch=3)
    spec, n = co.layout(net.channels, net.hidden, net.outputs)
    p = co.he_init(spec, n, 3)
    rng = np.random.default_rng(layer)
    o, nb = spec[layer]["b"]
    p[o:o + nb] = rng.normal(0, 0.1, nb)
    net.set_params(p)
    x = rng.normal(size=(3, H, H, cin))
    xg = bf16_tensor(torch, x).contiguous()
    out = torch.empty((3, H, H, cout), dtype=torch.bfloat16, device="cuda:0")
    net.conv_forward(layer, xg, out)
    net.synchronize()
    got = out.float().cpu().numpy()
    sp = spec[layer]
    w = co.bf16_round(p[sp["w"][0]:sp["w"][0] + sp["w"][1]].reshape(sp["shape"]))
    ref = np.maximum(co.conv3x3(co.bf16_round(x), w, p[sp["b"][0]:sp["b"][0] + sp["b"][1]]), 0)
    # FP32 accumulation then one bfloat16 rounding of the output
    err = np.abs(got - ref)
    assert np.all(err <= 2.0 ** -8 * np.abs(ref) + 1e-4 * np.abs(ref).max())


def test_forward_and_gradients_match_oracle(torch_cnn):
    torch, cnn = torch_cnn
    say("full network 32x32 batch 4: forward, loss, gradients vs oracle")
    net = cnn.Network(size=32, batch=4, outputs=5, hidden=16)
    m = co.Model(net.channels, net.hidden, net.outputs, bf16=True)
    p = co.he_init(m.spec, m.n, 7)
    rng = np.random.default_rng(7)
    for sp in m.spec:
        o, nb = sp["b"]
        p[o:o + nb] = rng.normal(0, 0.05, nb)
    p32 = p.astype(np.float32).astype(np.float64)
    net.set_params(p32)
    imgs = (rng.random((4, 32, 32)) < 0.35).astype(np.uint8)
    tgt = rng.normal(size=(4, 5))
    x = torch.from_numpy(imgs).to("cuda:0")
    t = torch.from_numpy(tgt.astype(np.float32)).to("cuda:0")
    y = net.forward(x)
    loss = net.mse(t)
    net.backward()
    net.synchronize()
    yg = y.cpu().numpy().astype(np.float64)
    yo = m.forward(p32, imgs)
    lo, dy = co.mse(yo, tgt)
    go = m.backward(p32, dy)
    gg = net.grads().astype(np.float64)
    assert np.max(np.abs(yg - yo)) <= 0.02 * np.max(np.abs(yo)) + 1e-4
    assert float(loss.cpu()) == pytest.approx(lo, rel=0.02)
    cos = gg @ go / (np.linalg.norm(gg) * np.linalg.norm(go))
    rel = np.linalg.norm(gg - go) / np.linalg.norm(go)
    say(f"  gradient cosine {cos:.6f}, relative L2 error {rel:.2e}")
    assert cos > 0.999 and rel < 0.05
    # per layer: every layer's gradient agrees in direction
    for sp in m.spec:
        o, nw = sp["w"]
        a, b = gg[o:o + nw], go[o:o + nw]
        assert a @ b / (np.linalg.norm(a) * np.linalg.norm(b) + 1e-30) > 0.99


def test_forward_at_c5_size_matches_oracle(torch_cnn):
    # 128 x 128 images, the surrogate's size: layers 2-4 (64, 32, 16 pixels
    # square) run the staged-patch kernel with 8 x 16 tiles and pooling,
    # layer 5 (8 x 8) the staged kernel with 8 x 8 tiles and a plain store
    torch, cnn = torch_cnn
    say("full network 128x128 batch 3: forward vs oracle")
    net = cnn.Network(size=128, batch=3)
    m = co.Model(net.channels, net.hidden, net.outputs, bf16=True)
    p = co.he_init(m.spec, m.n, 11)
    rng = np.random.default_rng(11)
    for sp in m.spec:
        o, nb = sp["b"]
        p[o:o + nb] = rng.normal(0, 0.05, nb)
    p32 = p.astype(np.float32).astype(np.float64)
    net.set_params(p32)
    imgs = (rng.random((3, 128, 128)) < 0.35).astype(np.uint8)
    y = net.forward(torch.from_numpy(imgs).to("cuda:0"))
    net.synchronize()
    yg = y.cpu().numpy().astype(np.float64)
    yo = m.forward(p32, imgs)
    assert np.max(np.abs(yg - yo)) <= 0.02 * np.max(np.abs(yo)) + 1e-4


def test_adam_and_training_reduce_loss(torch_cnn):
    torch, cnn = torch_cnn
    say("training 200 steps on 64 images 32x32")
    net = cnn.Network(size=32, batch=16, outputs=3, hidden=32)
    spec, n = co.layout(net.channels, net.hidden, net.outputs)
    p0 = co.he_init(spec, n, 1)
    net.set_params(p0)
    # one Adam step agrees with the oracle's update of the GPU gradient
    rng = np.random.default_rng(1)
    imgs = (rng.random((64, 32, 32)) < 0.3).astype(np.uint8)
    frac = imgs.reshape(64, -1).mean(axis=1)
    tgt = np.stack([frac, frac ** 2, 1 - frac], axis=1).astype(np.float32)
    x = torch.from_numpy(imgs).to("cuda:0")
    t = torch.from_numpy(tgt).to("cuda:0")
    net.forward(x[:16]); net.mse(t[:16]); net.backward()
    g = net.grads().astype(np.float64)
    net.adam_step(1e-3)
    p1 = net.params().astype(np.float64)
    pe, _, _ = co.adam(p0.astype(np.float32).astype(np.float64), g, np.zeros(n), np.zeros(n),
                       1e-3, 0.9, 0.999, 1e-8, 1)
    assert np.max(np.abs(p1 - pe)) < 1e-6
    net.set_params(p0)
    first = None
    for it in range(200):
        i = (it * 16) % 64
        loss = float(net.train_step(x[i:i + 16], t[i:i + 16], 1e-3).cpu())
        first = loss if first is None else first
    say(f"  loss {first:.4f} -> {loss:.4f}")
    assert loss < 0.2 * first


def test_training_is_deterministic(torch_cnn):
    torch, cnn = torch_cnn
    say("two identical 20-step trainings")
    out = []
    for _ in range(2):
        net = cnn.Network(size=32, batch=8, outputs=2, hidden=16)
        spec, n = co.layout(net.channels, net.hidden, net.outputs)
        net.set_params(co.he_init(spec, n, 2))
        rng = np.random.default_rng(2)
        x = torch.from_numpy((rng.random((8, 32, 32)) < 0.5).astype(np.uint8)).to("cuda:0")
        t = torch.from_numpy(rng.normal(size=(8, 2)).astype(np.float32)).to("cuda:0")
        for _ in range(20):
            net.train_step(x, t, 1e-3)
        out.append(net.params())
    assert np.array_equal(out[0], out[1])

"""Kernel-by-kernel parity of the surrogate network at its production size.

One training pass (forward, loss, backward) of the 128 x 128 network runs
through the C ABI exactly as in training, so every production kernel path
runs: the fused first layer with pooling, the staged-patch convolutions
with the pooling epilogue (layers 1-3) and the plain store (layer 4), global
average pooling, the dense layers, the loss, the input gradients on the
staged kernels with the raw and expanding epilogues and on the direct
kernel (layer 4), the weight gradients with their split sums, and the first
layer's backward kernel.  Each kernel's output is then checked against the
FP64 oracle evaluated on that kernel's own inputs as the GPU stored them
(BF16 activations and weights, FP32 elsewhere), so errors do not compound
from layer to layer.

The bar: a result the GPU rounds to BF16 must lie between the oracle's
value rounded the same way from v - e and from v + e, where v is the exact
(FP64) sum and e the worst-case FP32 accumulation error (K + 2) 2^-24 sum|terms|
of its K terms, and at least 99 % of them must equal the oracle's value of
the exact sum rounded the same way bit for bit (FP32 accumulation can only
move a result across a BF16 rounding boundary when the exact sum lies within
e of it).  FP32 results lie within e of v, where weight
gradients, summed over K pixels in MFMA steps of 32 and split partials,
take e = (K / 32 + 64) 2^-24 sum|terms|.
"""
import sys

import numpy as np
import pytest

from oracle import cnn_oracle as co

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
B = 4
# 128 x 128 images (the benchmark's) and 64 x 64 (the small surrogate
# test's): the sizes select different kernels (8 x 16 / 8 x 32 tiles, the
# row-walking or the strided first-layer backward, direct kernels for the
# 4 x 4 last layer)
SIZES = (128, 64)


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def bf(a):
    return co.bf16_round(a)


def relu(a):
    return np.maximum(a, 0.0)


def pooled_bf16(q):
    """The pooling epilogue on BF16 ReLU outputs q [N, H, W, C]: FP32 sum of
    the quad in the order (0,0) (0,1) (1,0) (1,1), times 0.25, to BF16."""
    q = q.astype(np.float32)
    s = np.zeros((q.shape[0], q.shape[1] // 2, q.shape[2] // 2, q.shape[3]), np.float32)
    for dy, dx in ((0, 0), (0, 1), (1, 0), (1, 1)):
        s = s + q[:, dy::2, dx::2, :]
    return bf(np.float32(0.25) * s)


def check_between(got, lo, hi, what, exact=None, min_equal=0.99):
    """Every value inside its rigorous bound [lo, hi]; where `exact` (the
    oracle's value of the exact sum, rounded as the GPU rounds) is given, at
    least `min_equal` of the values equal it bit for bit."""
    got = np.asarray(got, np.float64)
    bad = (got < lo) | (got > hi)
    assert not bad.any(), (f"{what}: {int(bad.sum())} of {got.size} outside the bounds, e.g. "
                           f"{got[bad][:3]} not in [{lo[bad][:3]}, {hi[bad][:3]}]")
    msg = f"  {what}: {got.size} values within bounds"
    if exact is not None:
        eq = np.mean(got == exact)
        msg += f", {100 * eq:.3f} % bitwise equal to the rounded exact value"
    say(msg)
    if exact is not None:
        assert eq >= min_equal


def check_close(got, ref, err, what):
    got = np.asarray(got, np.float64)
    d = np.abs(got - ref)
    bad = d > err
    assert not bad.any(), (f"{what}: {int(bad.sum())} of {got.size} beyond the FP32 bound, worst "
                           f"{np.max(d - err):.3e}")
    say(f"  {what}: {got.size} values, largest error {np.max(d / np.maximum(err, 1e-300)):.2f} of the bound")


def conv_bounds(x, w, b):
    """Exact conv (ReLU not applied) and its FP32 accumulation bound."""
    K = 9 * x.shape[3]
    v = co.conv3x3(x, w, b)
    s = co.conv3x3(np.abs(x), np.abs(w), np.abs(b))
    return v, (K + 2) * U * s


@pytest.fixture(scope="module", params=SIZES, ids=lambda s: f"{s}px")
def run(request):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_04565_amd import cnn
    SIZE = request.param
    say(f"surrogate network {SIZE}x{SIZE}, batch {B}: one forward + loss + backward")
    net = cnn.Network(size=SIZE, batch=B)
    spec, n = co.layout(net.channels, net.hidden, net.outputs)
    rng = np.random.default_rng(21)
    p = co.he_init(spec, n, 21)
    for sp in spec:
        o, nb = sp["b"]
        p[o:o + nb] = rng.normal(0, 0.05, nb)
    p = p.astype(np.float32).astype(np.float64)
    net.set_params(p)
    from paper_2201_04565_amd import inputs
    imgs = np.stack([inputs.circular_inclusions(SIZE, seed=500 + i) for i in range(B)])
    tgt = rng.normal(size=(B, net.outputs)).astype(np.float32)
    x = torch.from_numpy(imgs).to("cuda:0")
    t = torch.from_numpy(tgt).to("cuda:0")
    net.forward(x)
    net.mse(t)
    net.backward()
    net.synchronize()
    H = [SIZE >> l for l in range(5)]
    C = [1] + list(net.channels)
    buf = {}
    for l in range(4):
        buf["pooled", l] = net.buffer("pooled", l).astype(np.float64).reshape(B, H[l] // 2, H[l] // 2, C[l + 1])
    for l in range(1, 4):
        buf["mask", l] = net.buffer("mask", l).reshape(B, H[l] // 2, H[l] // 2, C[l + 1])
    for l in range(1, 5):
        buf["dact", l] = net.buffer("dact", l).astype(np.float64).reshape(B, H[l], H[l], C[l + 1])
    buf["act"] = net.buffer("act").astype(np.float64).reshape(B, H[4], H[4], C[5])
    buf["dpool0"] = net.buffer("dpool0").astype(np.float64).reshape(B, H[0] // 2, H[0] // 2, C[1])
    for nm in ("gap", "dgap", "hidden", "dhidden", "out", "dout"):
        buf[nm] = net.buffer(nm).astype(np.float64).reshape(B, -1)
    g = net.grads().astype(np.float64)

    def W(l, bf16=True):
        sp = spec[l]
        w = p[sp["w"][0]:sp["w"][0] + sp["w"][1]].reshape(sp["shape"])
        return (bf(w) if bf16 else w), p[sp["b"][0]:sp["b"][0] + sp["b"][1]]

    def G(l):
        sp = spec[l]
        return (g[sp["w"][0]:sp["w"][0] + sp["w"][1]].reshape(sp["shape"]),
                g[sp["b"][0]:sp["b"][0] + sp["b"][1]])

    return dict(imgs=imgs.astype(np.float64)[..., None], tgt=tgt, buf=buf, W=W, G=G, H=H, C=C)


def test_forward_first_layer_pooled(run):
    b, (w, bias) = run["buf"], run["W"](0, bf16=False)  # FP32 weights on the vector units
    v = co.conv3x3(run["imgs"], w, bias)
    e = 12 * U * co.conv3x3(run["imgs"], np.abs(w), np.abs(bias))
    check_between(b["pooled", 0], pooled_bf16(bf(relu(v - e))), pooled_bf16(bf(relu(v + e))),
                  "layer 0 conv + ReLU + pool (VALU)", exact=pooled_bf16(bf(relu(v))))


@pytest.mark.parametrize("l", [1, 2, 3])
def test_forward_pooled_layers(run, l):
    b, (w, bias) = run["buf"], run["W"](l)
    v, e = conv_bounds(b["pooled", l - 1], w, bias)
    check_between(b["pooled", l], pooled_bf16(bf(relu(v - e))), pooled_bf16(bf(relu(v + e))),
                  f"layer {l} staged conv + pooling epilogue", exact=pooled_bf16(bf(relu(v))))
    # ReLU mask: bit d of a pooled pixel is the sign of the conv output at
    # quad position d = 2 dy + dx; it may differ only where |v| <= e
    m = b["mask", l]
    for d, (dy, dx) in enumerate(((0, 0), (0, 1), (1, 0), (1, 1))):
        bit = (m >> d) & 1
        vv, ee = v[:, dy::2, dx::2, :], e[:, dy::2, dx::2, :]
        assert np.all(bit[vv - ee > 0] == 1) and np.all(bit[vv + ee <= 0] == 0)


def test_forward_last_conv(run):
    b, (w, bias) = run["buf"], run["W"](4)
    v, e = conv_bounds(b["pooled", 3], w, bias)
    check_between(b["act"], bf(relu(v - e)), bf(relu(v + e)), "layer 4 staged conv, plain store",
                  exact=bf(relu(v)))


def test_forward_pooling_and_dense(run):
    b = run["buf"]
    act = b["act"].reshape(B, -1, run["C"][5])
    HW = act.shape[1]
    check_close(b["gap"], act.sum(axis=1) / HW, (HW + 2) * U * np.abs(act).sum(axis=1) / HW,
                "global average pooling")
    for x, (w, bias), nm, outn, r in ((b["gap"], run["W"](5, False), "dense 0 + ReLU", "hidden", True),
                                      (b["hidden"], run["W"](6, False), "dense 1", "out", False)):
        v = co.dense(x, w, bias)
        e = (x.shape[1] + 2) * U * co.dense(np.abs(x), np.abs(w), np.abs(bias))
        lo, hi = (relu(v - e), relu(v + e)) if r else (v - e, v + e)
        check_between(b[outn], lo, hi, nm)


def test_loss_gradient(run):
    b = run["buf"]
    n = b["out"].size
    ref = 2.0 * (b["out"] - run["tgt"]) / n
    check_close(b["dout"], ref, 4 * U * np.abs(ref) + 1e-30, "mean squared error gradient")


def test_backward_dense_and_gap(run):
    b = run["buf"]
    w1, _ = run["W"](6, False)
    w0, _ = run["W"](5, False)
    dy, h1, g0 = b["dout"], b["hidden"], b["gap"]
    # weight and bias gradients of both dense layers (sums over the batch)
    for (gw, gb), dout, xin, nm in ((run["G"](6), dy, h1, "dense 1"), (run["G"](5), b["dhidden"], g0, "dense 0")):
        check_close(gw, dout.T @ xin, (B + 2) * U * (np.abs(dout).T @ np.abs(xin)), f"{nm} weight gradient")
        check_close(gb, dout.sum(axis=0), (B + 2) * U * np.abs(dout).sum(axis=0), f"{nm} bias gradient")
    v = (dy @ w1) * (h1 > 0)
    check_close(b["dhidden"], v, (w1.shape[0] + 2) * U * (np.abs(dy) @ np.abs(w1)), "dense 1 input gradient")
    v = b["dhidden"] @ w0
    check_close(b["dgap"], v, (w0.shape[0] + 2) * U * (np.abs(b["dhidden"]) @ np.abs(w0)),
                "dense 0 input gradient")
    # conv-output gradient of the last layer: dgap / HW where the ReLU passed,
    # an exact division by a power of two, then BF16 -- bit for bit
    HW = b["act"].shape[1] * b["act"].shape[2]
    dg = b["dgap"].astype(np.float32) / np.float32(HW)
    ref = bf(np.broadcast_to(dg[:, None, None, :], b["act"].shape)) * (b["act"] > 0)
    assert np.array_equal(b["dact", 4], ref)


@pytest.mark.parametrize("l", [1, 2, 3, 4])
def test_weight_gradients(run, l):
    b = run["buf"]
    xin, dout = b["pooled", l - 1], b["dact", l]
    w, _ = run["W"](l)
    _, dw, db = co.conv3x3_backward(xin, w, dout)
    _, sw, sb = co.conv3x3_backward(np.abs(xin), np.abs(w), np.abs(dout))
    K = dout.shape[0] * dout.shape[1] * dout.shape[2]
    gw, gb = run["G"](l)
    c = (K / 32 + 64) * U
    check_close(gw, dw, c * sw, f"layer {l} weight gradient (MFMA, {K} pixels, split sums)")
    check_close(gb, db, c * sb, f"layer {l} bias gradient")


@pytest.mark.parametrize("l", [2, 3, 4])
def test_input_gradients_expanding(run, l):
    # gradient of layer l's input (the pooled map of layer l - 1) written at
    # the full resolution of layer l - 1: 0.25 bf16(dx) where the ReLU mask
    # of layer l - 1 is set, 0 elsewhere
    b = run["buf"]
    w, _ = run["W"](l)
    dx, _, _ = co.conv3x3_backward(b["pooled", l - 1], w, b["dact", l])
    sx, _, _ = co.conv3x3_backward(b["pooled", l - 1], np.abs(w), np.abs(b["dact", l]))
    e = (9 * w.shape[0] + 2) * U * sx
    m = b["mask", l - 1]
    got = b["dact", l - 1]
    lo, hi = 0.25 * bf(dx - e), 0.25 * bf(dx + e)
    for d, (dy_, dx_) in enumerate(((0, 0), (0, 1), (1, 0), (1, 1))):
        on = ((m >> d) & 1).astype(bool)
        gq = got[:, dy_::2, dx_::2, :]
        assert np.all(gq[~on] == 0.0)
        check_between(gq[on], lo[on], hi[on], f"layer {l} input gradient, expanding epilogue, position {d}",
                      exact=(0.25 * bf(dx))[on])


def test_input_gradient_raw(run):
    b = run["buf"]
    w, _ = run["W"](1)
    dx, _, _ = co.conv3x3_backward(b["pooled", 0], w, b["dact", 1])
    sx, _, _ = co.conv3x3_backward(b["pooled", 0], np.abs(w), np.abs(b["dact", 1]))
    e = (9 * w.shape[0] + 2) * U * sx
    check_between(b["dpool0"], bf(dx - e), bf(dx + e), "layer 1 input gradient, raw epilogue",
                  exact=bf(dx))


def test_first_layer_backward(run):
    # the first layer's backward kernel takes the ReLU signs of its conv
    # outputs (FP32 from the image) kept by the forward pass and sums the tap and bias gradients
    # of the pooled gradient; signs within the FP32 error of zero may go
    # either way and widen the bound by their terms
    b = run["buf"]
    x = run["imgs"]
    w, bias = run["W"](0, bf16=False)
    v = co.conv3x3(x, w, bias)
    ev = 12 * U * co.conv3x3(x, np.abs(w), np.abs(bias))
    up = co.pool2_backward(b["dpool0"])
    sure = (v - ev > 0).astype(np.float64)
    amb = (np.abs(v) <= ev).astype(np.float64)
    _, dw, db = co.conv3x3_backward(x, w, up * sure)
    _, sw, sb = co.conv3x3_backward(x, w, np.abs(up))
    _, aw, ab = co.conv3x3_backward(x, w, np.abs(up) * amb)
    K = up.shape[0] * up.shape[1] * up.shape[2]
    gw, gb = run["G"](0)
    c = (K / 32 + 64) * U
    say(f"  {int(amb.sum())} conv outputs of the first layer within FP32 error of zero")
    check_close(gw, dw, c * sw + aw, f"layer 0 weight gradient ({K} pixels)")
    check_close(gb, db, c * sb + ab, "layer 0 bias gradient")

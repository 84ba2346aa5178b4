"""FP64 reference of the surrogate network (test infrastructure only).

Plain numpy, direct definitions: 3x3 convolution with zero padding, ReLU,
2x2 average pooling, global average pooling, dense layers, mean squared
error and their gradients, and the Adam update.  Only the tests use it.

Parameter vector layout (shared with the GPU library as a definition, not
code): for each conv layer the weights [Cout][3][3][Cin] then the bias
[Cout]; then each dense layer's weights [out][in] and bias [out].

`bf16=True` rounds weights and activations to bfloat16 (round to nearest
even) at the points where the GPU stores them in that format: conv weights,
conv outputs after ReLU, pooled maps, and the gradients of those maps.
Parity unpinned: nothing here; the functions are pinned by
`tests/test_oracle_cnn.py` (closed forms, finite differences).
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """Round to bfloat16 (nearest even) and return as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def layout(channels, hidden, outputs, in_channels=1):
    """Offsets of each layer's weights and bias in the parameter vector."""
    out = []
    o = 0
    cin = in_channels
    for c in channels:
        nw = c * 9 * cin
        out.append(dict(kind="conv", w=(o, nw), b=(o + nw, c), shape=(c, 3, 3, cin)))
        o += nw + c
        cin = c
    for i, (nin, nout) in enumerate(((cin, hidden), (hidden, outputs))):
        nw = nout * nin
        out.append(dict(kind="dense", w=(o, nw), b=(o + nw, nout), shape=(nout, nin)))
        o += nw + nout
    return out, o


def _get(params, spec, key):
    off, n = spec[key]
    return params[off:off + n]


# ------------------------------------------------------------------ layers
def conv3x3(x, w, b):
    """x [N,H,W,Cin], w [Cout,3,3,Cin], b [Cout] -> [N,H,W,Cout]; zero pad."""
    N, H, W, _ = x.shape
    xp = np.zeros((N, H + 2, W + 2, x.shape[3]))
    xp[:, 1:-1, 1:-1, :] = x
    y = np.zeros((N, H, W, w.shape[0]))
    for ky in range(3):
        for kx in range(3):
            y += np.einsum("nhwc,oc->nhwo", xp[:, ky:ky + H, kx:kx + W, :], w[:, ky, kx, :])
    return y + b


def conv3x3_backward(x, w, dy):
    """Gradients of conv3x3 wrt x, w and b for output gradient dy."""
    N, H, W, Cin = x.shape
    xp = np.zeros((N, H + 2, W + 2, Cin))
    xp[:, 1:-1, 1:-1, :] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            dw[:, ky, kx, :] = np.einsum("nhwo,nhwc->oc", dy, xp[:, ky:ky + H, kx:kx + W, :])
            dxp[:, ky:ky + H, kx:kx + W, :] += np.einsum("nhwo,oc->nhwc", dy, w[:, ky, kx, :])
    return dxp[:, 1:-1, 1:-1, :], dw, dy.sum(axis=(0, 1, 2))


def pool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def gap(x):
    return x.mean(axis=(1, 2))


def gap_backward(dy, shape):
    N, H, W, C = shape
    return np.broadcast_to(dy[:, None, None, :] / (H * W), shape).copy()


def dense(x, w, b):
    return x @ w.T + b


# ------------------------------------------------------------------- model
class Model:
    def __init__(self, channels, hidden, outputs, bf16=False):
        self.channels = list(channels)
        self.spec, self.n = layout(channels, hidden, outputs)
        self.bf16 = bf16

    def _r(self, a):
        return bf16_round(a) if self.bf16 else a

    def forward(self, params, images):
        """images [N,H,W] (phase 0/1) -> outputs [N, outputs]; keeps a tape."""
        x = np.asarray(images, dtype=np.float64)[..., None]
        tape = dict(x=x, acts=[], pools=[])
        h = x
        nconv = len(self.channels)
        for l in range(nconv):
            sp = self.spec[l]
            w = _get(params, sp, "w").reshape(sp["shape"])
            if l > 0:
                w = self._r(w)          # conv weights are BF16 on the matrix cores
            a = self._r(np.maximum(conv3x3(h, w, _get(params, sp, "b")), 0.0))
            tape["acts"].append(a)
            if l < nconv - 1:
                h = self._r(pool2(a))
                tape["pools"].append(h)
        g = gap(tape["acts"][-1])
        d1, d2 = self.spec[nconv], self.spec[nconv + 1]
        h1 = np.maximum(dense(g, _get(params, d1, "w").reshape(d1["shape"]), _get(params, d1, "b")), 0.0)
        y = dense(h1, _get(params, d2, "w").reshape(d2["shape"]), _get(params, d2, "b"))
        tape.update(g=g, h1=h1)
        self.tape = tape
        return y

    def backward(self, params, dy):
        """Gradient of the parameters for output gradient dy (after forward)."""
        t = self.tape
        grad = np.zeros(self.n)
        nconv = len(self.channels)
        d1, d2 = self.spec[nconv], self.spec[nconv + 1]
        w2 = _get(params, d2, "w").reshape(d2["shape"])
        w1 = _get(params, d1, "w").reshape(d1["shape"])
        o, n = d2["w"]
        grad[o:o + n] = (dy.T @ t["h1"]).ravel()
        o, n = d2["b"]
        grad[o:o + n] = dy.sum(axis=0)
        dh1 = (dy @ w2) * (t["h1"] > 0)
        o, n = d1["w"]
        grad[o:o + n] = (dh1.T @ t["g"]).ravel()
        o, n = d1["b"]
        grad[o:o + n] = dh1.sum(axis=0)
        dg = dh1 @ w1
        acts = t["acts"]
        da = self._r(gap_backward(dg, acts[-1].shape) * (acts[-1] > 0))
        for l in range(nconv - 1, -1, -1):
            sp = self.spec[l]
            w = _get(params, sp, "w").reshape(sp["shape"])
            if l > 0:
                w = self._r(w)
            xin = t["pools"][l - 1] if l > 0 else t["x"]
            dx, dw, db = conv3x3_backward(xin, w, da)
            o, n = sp["w"]
            grad[o:o + n] = dw.ravel()
            o, n = sp["b"]
            grad[o:o + n] = db
            if l > 0:
                dpool = self._r(dx)
                da = self._r(pool2_backward(dpool) * (acts[l - 1] > 0))
        return grad


def mse(y, target):
    d = y - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam(p, g, m, v, lr, b1, b2, eps, t):
    """One Adam step (bias-corrected moments); returns new p, m, v."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def he_init(spec, n, seed):
    """He-normal weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(n)
    for sp in spec:
        o, nw = sp["w"]
        fan_in = int(np.prod(sp["shape"][1:]))
        p[o:o + nw] = rng.normal(0.0, np.sqrt(2.0 / fan_in), nw)
    return p

"""Surrogate pipeline: batched lattice spring model labels, an ensemble of
CNNs trained on them, and an uncertainty gate that falls back to the model.

* labels: 64-point sigma_xx curve (one point per 0.5 % strain increment)
  and the modulus of each specimen, from `lsm.Batch` runs to the increment
  cap;
* training: K networks (`cnn.Network`, BF16 matrix-core kernels) with
  different initialisations and data orders, Adam, standardised targets;
* inference: the ensemble mean; a specimen whose predicted moduli spread
  (std / mean over the members) exceeds the gate is sent to the batched
  model instead, so every accepted answer carries the ensemble's agreement.

The lattice spring model is both the fallback and the reference for the
surrogate's error (the paper motivates the code by fast data generation
for machine-learning materials design: Abstract, Section 4).
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import cnn, inputs, lsm

CURVE_POINTS = 64
SIZE = 128


def specimen_images(n: int, seed0: int, size: int = SIZE) -> np.ndarray:
    """Circular-inclusion images of one side (seed seed0 + i)."""
    return np.stack([inputs.circular_inclusions(size, seed=seed0 + i) for i in range(n)])


@dataclass
class Labels:
    curves: np.ndarray    # [n, 64] sigma_xx per increment
    modulus: np.ndarray   # [n]
    strength: np.ndarray  # [n]
    seconds: float        # GPU wall time of the batched runs


def label(images: np.ndarray, chunk: int = 8192, steps: int = 500, d_eps: float = 0.005,
          device: str = "cuda:0", log=None) -> Labels:
    """Runs the batched model on every image to CURVE_POINTS increments."""
    import torch

    wl = dict(inputs.WORKLOADS["c4"])
    cur, mod, st = [], [], []
    secs = 0.0
    for s in range(0, len(images), chunk):
        b = lsm.Batch.from_workload(wl, list(images[s:s + chunk]), precision="fp32k", device=device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # drop 0: every specimen runs to the cap, giving full-length curves
        b.run(d_eps, steps, CURVE_POINTS, drop=0.0)
        torch.cuda.synchronize()
        secs += time.perf_counter() - t0
        r = b.read()
        if log is not None:
            log(f"labelled {min(s + chunk, len(images))}/{len(images)} specimens ({secs:.1f} s)")
        cur.append(r["sigma_xx"])
        mod.append(r["modulus"])
        st.append(r["strength"])
        del b
        torch.cuda.empty_cache()
    return Labels(np.concatenate(cur), np.concatenate(mod), np.concatenate(st), secs)


def targets(lab: Labels) -> np.ndarray:
    return np.concatenate([lab.curves, lab.modulus[:, None]], axis=1).astype(np.float64)


def _he_normal(net: cnn.Network, seed: int) -> np.ndarray:
    """He-normal weights, zero biases, seeded."""
    wo, bo, wn = net.layout()
    rng = np.random.default_rng(seed)
    p = np.zeros(net.n_params, np.float32)
    fan = [9 * c for c in (1,) + net.channels[:-1]] + [net.channels[-1], net.hidden]
    for l in range(7):
        p[wo[l]:wo[l] + wn[l]] = rng.normal(0.0, np.sqrt(2.0 / fan[l]), wn[l])
    return p


class Surrogate:
    """K networks; mean prediction and modulus spread."""

    def __init__(self, k: int = 5, size: int = SIZE, batch: int = 512,
                 outputs: int = CURVE_POINTS + 1, device: str = "cuda:0", seed: int = 0,
                 modulus_weight: float = 4.0):
        import torch

        self.torch = torch
        self.k, self.batch, self.device = k, batch, device
        # the modulus is one output of 65: scaling its standardised target by
        # w weights it w^2 in the mean squared error
        self.modulus_weight = modulus_weight
        self.nets = [cnn.Network(size=size, batch=batch, outputs=outputs, device=device)
                     for _ in range(k)]
        for i, n in enumerate(self.nets):
            n.set_params(_he_normal(n, seed * 1000 + i))
        self.mu = None
        self.sd = None
        self.train_seconds = 0.0
        self.train_flops = 0.0

    def fit(self, images: np.ndarray, y: np.ndarray, epochs: int = 20, lr: float = 2e-3,
            seed: int = 0, log=None):
        torch = self.torch
        self.mu = y.mean(axis=0)
        self.sd = y.std(axis=0) + 1e-12
        self.sd[-1] /= self.modulus_weight
        x = torch.from_numpy(np.ascontiguousarray(images)).to(self.device)
        t = torch.from_numpy(((y - self.mu) / self.sd).astype(np.float32)).to(self.device)
        n = len(images)
        B = self.batch
        steps_per_epoch = n // B
        total = steps_per_epoch * epochs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, net in enumerate(self.nets):
            rng = np.random.default_rng(seed * 7919 + i)
            it = 0
            for ep in range(epochs):
                order = torch.from_numpy(rng.permutation(n)).to(self.device)
                for s in range(steps_per_epoch):
                    idx = order[s * B:(s + 1) * B]
                    xb = x.index_select(0, idx).contiguous()
                    tb = t.index_select(0, idx).contiguous()
                    # cosine learning-rate decay
                    lr_it = 0.5 * lr * (1.0 + np.cos(np.pi * it / max(total, 1)))
                    loss = net.train_step(xb, tb, lr_it)
                    it += 1
                if log is not None:
                    net.synchronize()
                    log(f"member {i} epoch {ep}: loss {float(loss.cpu()):.4f}")
        for net in self.nets:
            net.synchronize()
        torch.cuda.synchronize()
        self.train_seconds = time.perf_counter() - t0
        return self

    def predict(self, images: np.ndarray, repeats: int = 1):
        """Returns (mean prediction [n, outputs], modulus spread [n], seconds).

        With repeats > 1 the ensemble runs once untimed and then `repeats`
        times timed (the same outputs each time); seconds is the median."""
        torch = self.torch
        x = torch.from_numpy(np.ascontiguousarray(images)).to(self.device)
        n = len(images)
        outs = np.zeros((self.k, n, len(self.mu)))
        times = []
        for rep in range(repeats + 1 if repeats > 1 else 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            dev_outs = [[] for _ in range(self.k)]
            for s in range(0, n, self.batch):
                xb = x[s:s + self.batch].contiguous()
                for i, net in enumerate(self.nets):
                    dev_outs[i].append(net.forward(xb).clone())
            for net in self.nets:
                net.synchronize()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        secs = float(np.median(times[1:] if repeats > 1 else times))
        for i in range(self.k):
            outs[i] = torch.cat(dev_outs[i]).cpu().numpy() * self.sd + self.mu
        mean = outs.mean(axis=0)
        mod = outs[:, :, -1]
        spread = mod.std(axis=0) / np.maximum(np.abs(mod.mean(axis=0)), 1e-12)
        return mean, spread, secs


def curve_strength(pred: np.ndarray) -> np.ndarray:
    return pred[:, :CURVE_POINTS].max(axis=1)


def calibrate_gate(sur: Surrogate, images: np.ndarray, lab: Labels, target_p95: float = 0.05,
                   max_gate: float = 0.05, min_accept: int = 20) -> dict:
    """Spread gate from a held-out split: the largest threshold (at most
    max_gate) whose accepted specimens -- spread at or below it, at least
    min_accept of them -- have a 95th-percentile modulus error within
    target_p95 on that split.  (The 95th percentile of fewer than 20 errors
    is their largest or second largest: a gate set on so few would not hold
    on another split.)  A gate of 0 sends every specimen to the model."""
    pred, spread, _ = sur.predict(images)
    err = np.abs(pred[:, -1] - lab.modulus) / np.abs(lab.modulus)
    order = np.argsort(spread, kind="stable")
    best = 0.0
    for m in range(1, len(order) + 1):
        g = float(spread[order[m - 1]])
        if g > max_gate:
            break
        if m >= min_accept and np.quantile(err[order[:m]], 0.95) <= target_p95:
            best = g
    acc = spread <= best
    return dict(gate=best, val_n=len(images), val_accept_rate=float(acc.mean()),
                val_accepted_p95=float(np.quantile(err[acc], 0.95)) if acc.any() else 0.0)


@dataclass
class Answers:
    """The pipeline's answer per specimen: the ensemble's, or the model's
    where the gate sent the specimen back to it."""
    modulus: np.ndarray
    strength: np.ndarray
    curves: np.ndarray
    fallback: np.ndarray          # bool per specimen
    spread: np.ndarray
    inference_s: float
    fallback_s: float
    fallback_labels: Labels | None


def answer(sur: Surrogate, images: np.ndarray, gate: float, steps: int = 500, d_eps: float = 0.005,
           repeats: int = 1) -> Answers:
    """Gated inference: the ensemble mean where its modulus spread is at or
    below the gate, the batched model's run of the specimen otherwise."""
    pred, spread, t_inf = sur.predict(images, repeats=repeats)
    fb = spread > gate
    mod = pred[:, -1].copy()
    cur = pred[:, :CURVE_POINTS].copy()
    stg = curve_strength(pred)
    fb_lab, t_fb = None, 0.0
    if fb.any():
        fb_lab = label(images[fb], steps=steps, d_eps=d_eps)
        t_fb = fb_lab.seconds
        mod[fb] = fb_lab.modulus
        stg[fb] = fb_lab.strength
        cur[fb] = fb_lab.curves
    return Answers(mod, stg, cur, fb, spread, t_inf, t_fb, fb_lab)


def evaluate(sur: Surrogate, images: np.ndarray, lab: Labels, gate: float = 0.05,
             steps: int = 500, d_eps: float = 0.005) -> dict:
    """Gated pipeline on a test split, scored against the model's own labels.

    Specimens whose ensemble spread exceeds the gate are re-run on the
    batched model and answered by it; the others keep the surrogate's
    prediction.  Throughput counts the surrogate inference (median of five
    timed passes after an untimed one) plus the fallback runs."""
    a = answer(sur, images, gate, steps, d_eps, repeats=5)
    pred, _, _ = sur.predict(images)
    err_sur = np.abs(pred[:, -1] - lab.modulus) / np.abs(lab.modulus)
    err_str_sur = np.abs(curve_strength(pred) - lab.strength) / np.abs(lab.strength)
    err = np.abs(a.modulus - lab.modulus) / np.abs(lab.modulus)
    err_str = np.abs(a.strength - lab.strength) / np.abs(lab.strength)
    acc = ~a.fallback
    n = len(images)
    return dict(
        n=n, gate=gate, fallback_rate=float(a.fallback.mean()),
        surrogate_modulus_err_mean=float(err_sur.mean()),
        surrogate_modulus_err_p95=float(np.quantile(err_sur, 0.95)),
        surrogate_strength_err_mean=float(err_str_sur.mean()),
        pipeline_modulus_err_mean=float(err.mean()),
        pipeline_modulus_err_p95=float(np.quantile(err, 0.95)),
        pipeline_strength_err_mean=float(err_str.mean()),
        accepted_modulus_err_p95=float(np.quantile(err[acc], 0.95)) if acc.any() else 0.0,
        accepted_modulus_err_max=float(err[acc].max()) if acc.any() else 0.0,
        inference_s=a.inference_s, fallback_s=a.fallback_s,
        specimens_per_hour=n / (a.inference_s + a.fallback_s) * 3600.0,
    )


def amortized(res: dict, label_s: float, train_s: float, model_s_per_specimen: float) -> dict:
    """Whole-pipeline cost including the labelling and training that built
    the surrogate: specimens/hour over N specimens, and the N from which
    the pipeline beats the batched model alone."""
    per = (res["inference_s"] + res["fallback_s"]) / res["n"]
    fixed = label_s + train_s
    gain = model_s_per_specimen - per
    be = fixed / gain if gain > 0 else float("inf")
    out = {"fixed_s": fixed, "per_specimen_s": per, "break_even_specimens": be}
    for N in (10 ** 5, 10 ** 6, 10 ** 7):
        out[f"specimens_per_hour_at_{N}"] = N / (fixed + N * per) * 3600.0
    return out

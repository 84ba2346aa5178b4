"""Benchmark: spring-steps/s of the lattice spring model hot path on one GPU.

Workload: 2048 x 2048 brick-and-mortar image -> triangular lattice
(4,194,304 particles, 12,574,721 springs), FP32 forces with compensated FP32
displacements, displacement-controlled tension in increments of 0.05 %
strain, 2000 damped velocity Verlet steps per increment.  One bench "step"
is one loading increment: strain increment + step-0 force evaluation, 2000
fused step kernels (spring forces with critical-stretch breaking, force
accumulation, integration), end-of-increment reductions and the break log.

spring-steps/s = springs in the list (broken ones included, they are still
iterated) x timesteps / wall time.  The roofline object rates the dominant
kernel (the fused step) by its algorithmic bytes per launch over its
average duration measured with HIP events on the library's stream.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = ("spring-steps/s (% HBM roofline); specimens/hour batched+surrogate "
          "@≤5% error")
COUNTER_FILE = os.path.join(ROOT, "profiles", "c2_step_counters.json")
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-instructions/s
# (78.6 TFLOP/s of non-packed FP32 FMA)
VALU_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12
WORKLOAD_NAMES = {
    "c2": "c2 brick-and-mortar 2048x2048 triangular lattice, fp32 forces with compensated fp32 "
          "displacements, 0.05% strain increments x 2000 steps",
    "c3": "c3 256^3 simple-cubic voxel lattice from a thresholded Gaussian random field (40% solid, "
          "largest cluster), face + edge springs, fp32 forces with compensated fp32 displacements, "
          "0.05% strain increments x 2000 steps",
}
KERNEL_SRC = os.path.join(ROOT, "paper_2201_04565_amd", "csrc", "lsm_kernels.hip")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_counters(launch):
    """rocprofv3 counters of the C2 step kernel (HBM bytes and VALU
    instructions per launch) from the committed summary, or None when
    absent, taken on a different kernel source or another launch shape."""
    try:
        with open(COUNTER_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_src_sha256") != kernel_hash():
        return None
    want = {k: launch[k] for k in ("variant", "rows_per_wave", "prefetch")}
    if t.get("launch") != want:
        return None
    return t


def cpu_baseline(wl, img, steps: int):
    """The FP64 oracle, single thread, on one increment of the same lattice."""
    import oracle
    prm = oracle.Params(k=wl["k"], s=wl["s"], mass=wl["mass"], a=wl.get("a", 1.0),
                        k_face=wl.get("k_face", 1.0), k_diag=wl.get("k_diag", 1.0),
                        dt=wl["dt"], gamma=wl["gamma"], void_value=wl.get("void_value", -1))
    net = oracle.Net.lattice(img, prm)
    t0 = time.perf_counter()
    net.apply_increment(wl["d_eps"])
    net.relax(steps)
    dt = time.perf_counter() - t0
    return dict(value=net.m * steps / dt, unit="spring-steps/s", cores=1, kind="oracle",
                sample=f"full {'x'.join(str(d) for d in img.shape[::-1])} lattice, 1 increment x "
                       f"{steps} steps (+ step-0 evaluation), FP64, single thread, {dt:.1f} s")


def batched_c4(args, torch, inputs, lsm):
    """Specimens/hour of the batched path on the 4096-specimen inclusion
    workload, beside the same kernels run one specimen at a time and the
    oracle on the host, all under the same failure rule."""
    import numpy as np

    wl = inputs.WORKLOADS["c4"]
    imgs = inputs.batch_specimens(args.batch_n)
    sizes = np.array([im.shape[0] for im in imgs])
    b = lsm.Batch.from_workload(wl, imgs, precision="fp32k", device="cuda:0")
    tune = b.autotune(20)
    launch = b.launch()
    print(f"[bench] batch launch: {launch}", file=sys.stderr, flush=True)
    b.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(wl["d_eps"], wl["steps"], wl["max_inc"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, steps, site_steps = b.read_timing()
    res = b.read()
    n_inc = res["n_inc"]
    out = dict(workload=f"{len(imgs)} inclusion specimens, sides {sorted(set(sizes.tolist()))}, "
                        f"0.5% x {wl['steps']} steps to failure (cap {wl['max_inc']}), fp32",
               particles=b.n_particles, springs=b.n_springs, wall_s=wall,
               specimens_per_hour=len(imgs) / wall * 3600.0,
               mean_increments=float(n_inc.mean()),
               # algorithmic bytes per particle-step: 50 for the one-step kernel,
               # 51 per two steps for the two-step kernel
               step_graph_GBs=site_steps * (25.5 if launch["steps_per_launch"] == 2 else 50)
               / (ms * 1e-3) / 1e9,
               launch=launch,
               autotune_us_per_step={f"{v} {r}x{p}": round(us, 1) for v, r, p, us in tune})
    del b
    torch.cuda.empty_cache()
    # plain: the same kernels, one specimen at a time, on a stratified sample
    per_size = {}
    for L in sorted(set(sizes.tolist())):
        idx = [i for i in range(len(imgs)) if sizes[i] == L][: args.plain_per_size]
        tt = []
        for i in idx:
            lat = lsm.Lattice.from_workload(wl, imgs[i], precision="fp32k", device="cuda:0")
            lat.synchronize()
            t1 = time.perf_counter()
            for _ in range(int(n_inc[i])):
                lat.apply_increment(wl["d_eps"])
                lat.relax(wl["steps"])
            lat.read_state()
            tt.append(time.perf_counter() - t1)
            del lat
        per_size[L] = float(np.mean(tt))
    plain_total = sum(per_size[int(L)] for L in sizes)
    out["plain_specimens_per_hour"] = len(imgs) / plain_total * 3600.0
    out["plain_sample"] = f"{args.plain_per_size} specimens per side, mean s/specimen {per_size}"
    out["batched_over_plain"] = out["specimens_per_hour"] / out["plain_specimens_per_hour"]
    return out


def cpu_c4(args, inputs):
    """Oracle on one host core: one specimen per side for a prefix of
    increments, extrapolated to the batch's increments (per-step cost is
    constant because broken springs stay in the list)."""
    import numpy as np

    import oracle
    wl = inputs.WORKLOADS["c4"]
    prm = oracle.Params(k=wl["k"], s=wl["s"], mass=wl["mass"], dt=wl["dt"], gamma=wl["gamma"])
    imgs = inputs.batch_specimens(args.batch_n)
    sizes = np.array([im.shape[0] for im in imgs])
    per_step = {}
    for L in sorted(set(sizes.tolist())):
        i = int(np.nonzero(sizes == L)[0][0])
        net = oracle.Net.lattice(imgs[i], prm)
        t0 = time.perf_counter()
        for _ in range(args.cpu_c4_inc):
            net.apply_increment(wl["d_eps"])
            net.relax(wl["steps"])
        per_step[L] = (time.perf_counter() - t0) / (args.cpu_c4_inc * wl["steps"])
    total = sum(per_step[int(L)] * wl["max_inc"] * wl["steps"] for L in sizes)
    return dict(value=len(imgs) / total * 3600.0, unit="specimens/hour", cores=1, kind="oracle",
                sample=f"one specimen per side, {args.cpu_c4_inc} increments each, "
                       f"extrapolated to {wl['max_inc']} increments per specimen")


def cnn_forward_flops(size=128, channels=(32, 64, 128, 128, 256), hidden=256, outputs=65):
    """Multiply-adds x 2 of one forward pass (convolutions and dense layers)."""
    f, cin, h = 0, 1, size
    for i, c in enumerate(channels):
        f += 2 * h * h * c * 9 * cin
        cin = c
        if i < len(channels) - 1:
            h //= 2
    return f + 2 * (cin * hidden + hidden * outputs)


def small_c1(args, inputs, lsm):
    """C1 (32 x 32 two-phase lattice, FP64, 20 x 0.5 % x 500 steps): a
    lattice this small is launch-bound, so the interior steps run in one
    workgroup with the state in LDS (one launch per relaxation chunk);
    timed beside per-step launches of the gather and two-step sweep
    kernels, with the oracle's full run on one host core."""
    wl = inputs.WORKLOADS["c1"]
    img = inputs.c1_image()
    res = {"workload": "c1 32x32 two-phase triangular lattice, fp64, 20 x 0.5% x 500 steps"}
    for variant in ("small", "gather", "sweep"):
        lat = lsm.Lattice.from_workload(wl, img, precision="fp64", device="cuda:0")
        lat.set_launch(variant)
        lat.apply_increment(wl["d_eps"])  # warm-up: graphs and code objects
        lat.relax(wl["steps"])
        lat.set_timing(True)
        lat.read_timing()
        lat.synchronize()
        t0 = time.perf_counter()
        for _ in range(wl["n_inc"] - 1):
            lat.apply_increment(wl["d_eps"])
            lat.relax(wl["steps"])
        lat.synchronize()
        wall = time.perf_counter() - t0
        ms, n = lat.read_timing()
        rec = lat.read_state()
        res[variant] = {"us_per_interior_step": 1e3 * ms / max(n, 1),
                        "steps_per_s_wall": (wl["n_inc"] - 1) * wl["steps"] / wall,
                        "broken_springs_at_end": rec["n_broken"]}
        del lat
    if not args.no_cpu:
        from oracle import Net, Params
        o = Net.lattice(img, Params(k=wl["k"], s=wl["s"], mass=wl["mass"], a=wl.get("a", 1.0),
                                    dt=wl["dt"], gamma=wl["gamma"], void_value=wl.get("void_value", -1)))
        t0 = time.perf_counter()
        for _ in range(wl["n_inc"]):
            o.apply_increment(wl["d_eps"])
            o.relax(wl["steps"])
        res["cpu_baseline"] = {"seconds_full_run": time.perf_counter() - t0, "cores": 1, "kind": "oracle",
                               "broken_springs_at_end": len(o.events())}
    return res


def cnn_kernels(torch, batch=512, size=128, iters=10):
    """Surrogate network kernels alone: one training step (forward, loss,
    backward, Adam) and one inference pass on a batch of 128 x 128 images,
    timed with events on the network's stream; rated against the BF16 dense
    matrix-core peak (2.5 PFLOP/s), a training step counted as 3 forwards."""
    import numpy as np

    from paper_2201_04565_amd import cnn, inputs
    from paper_2201_04565_amd.surrogate import _he_normal

    net = cnn.Network(size=size, batch=batch, outputs=65)
    net.set_params(_he_normal(net, 0))
    imgs = np.stack([inputs.circular_inclusions(size, seed=10 ** 7 + i) for i in range(batch)])
    x = torch.from_numpy(imgs).cuda()
    t = torch.from_numpy(np.random.default_rng(0).normal(size=(batch, 65)).astype(np.float32)).cuda()
    for _ in range(3):
        net.train_step(x, t, 1e-4)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(net.stream)
    for _ in range(iters):
        net.train_step(x, t, 1e-4)
    e1.record(net.stream)
    e1.synchronize()
    train_ms = e0.elapsed_time(e1) / iters
    e0.record(net.stream)
    for _ in range(iters):
        net.forward(x)
    e1.record(net.stream)
    e1.synchronize()
    fwd_ms = e0.elapsed_time(e1) / iters
    f = cnn_forward_flops(size) * batch
    return dict(batch=batch, size=size, train_step_ms=train_ms, forward_ms=fwd_ms,
                train_TFLOPs=3 * f / (train_ms * 1e-3) / 1e12,
                forward_TFLOPs=f / (fwd_ms * 1e-3) / 1e12,
                forward_frac_of_bf16_peak=f / (fwd_ms * 1e-3) / 2.5e15,
                inference_images_per_s=batch / (fwd_ms * 1e-3))


def surrogate_c5(args):
    """Batched model + surrogate pipeline on 128 x 128 inclusion specimens:
    labels from the batched model, a 5-member ensemble trained on them, a 5 %
    spread gate with fallback to the model; specimens/hour of the pipeline
    and of the batched model alone, and the modulus error against the
    model's own labels."""
    from paper_2201_04565_amd import surrogate as S

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    img_tr = S.specimen_images(args.sur_train, 10 ** 6)
    img_te = S.specimen_images(args.sur_test, 2 * 10 ** 6)
    log(f"images generated ({time.perf_counter() - t0:.1f} s)")
    lab_tr = S.label(img_tr, log=log)
    lab_te = S.label(img_te, log=log)
    sur = S.Surrogate(k=5, batch=512, seed=0)
    sur.fit(img_tr, S.targets(lab_tr), epochs=args.sur_epochs, lr=2e-3, log=log)
    res = S.evaluate(sur, img_te, lab_te, gate=0.05)
    res.update(
        workload=f"{args.sur_train} train / {args.sur_test} test 128x128 inclusion specimens, "
                 f"labels = 64-point sigma_xx curve + modulus (64 x 0.5% x 500 steps, fp32), "
                 f"5-member BF16 CNN ensemble, {args.sur_epochs} epochs, gate 5% spread",
        label_specimens_per_hour=len(img_tr) / lab_tr.seconds * 3600.0,
        batched_model_specimens_per_hour=len(img_te) / lab_te.seconds * 3600.0,
        train_s=sur.train_seconds,
        train_TFLOPs=3 * cnn_forward_flops() * 5 * args.sur_epochs * (len(img_tr) // 512) * 512
        / sur.train_seconds / 1e12,
        total_s=time.perf_counter() - t0)
    res["pipeline_over_batched_model"] = res["specimens_per_hour"] / res["batched_model_specimens_per_hour"]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("c2", "c3"), default="c2",
                    help="c2: 2048^2 brick-and-mortar (default); c3: 256^3 random-field voxels")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed loading increments (default 198 for c2, 5 for c3)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed loading increments")
    ap.add_argument("--steps-per-inc", type=int, default=None)
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kernel", choices=("auto", "sweep", "sweep2", "gather"), default="auto",
                    help="2D step kernel: auto (the two-step sweep), sweep (one step per launch), "
                         "sweep2 (two steps), gather (one thread per site)")
    ap.add_argument("--launch", default="0,1", metavar="ROWS,PREFETCH",
                    help="sweep launch: rows per wavefront (0: the library's occupancy-model "
                         "default), prefetch depth")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the launch with lsm_autotune instead of --launch")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched C4 measurement")
    ap.add_argument("--batch-n", type=int, default=4096)
    ap.add_argument("--plain-per-size", type=int, default=2)
    ap.add_argument("--cpu-c4-inc", type=int, default=1)
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the batched-model + surrogate pipeline (on by default at reduced size)")
    ap.add_argument("--cnn-bench", action="store_true", help="also time the surrogate network kernels")
    ap.add_argument("--no-c1", action="store_true", help="skip the small-lattice (C1) section")
    ap.add_argument("--sur-train", type=int, default=4096,
                    help="training specimens (the full C5 configuration: 50000)")
    ap.add_argument("--sur-test", type=int, default=1024, help="test specimens (C5: 5000)")
    ap.add_argument("--sur-epochs", type=int, default=10, help="epochs (C5: 20)")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (counter scale reference)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 198 if args.workload == "c2" else 5
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (a single "
              "lattice would shard as x-slabs with a halo exchange, a batch by specimen)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2201_04565_amd import inputs, lsm

    wl = inputs.WORKLOADS[args.workload]
    spi = args.steps_per_inc or wl["steps"]
    img = inputs.c2_image() if args.workload == "c2" else inputs.c3_image()
    lat = lsm.Lattice.from_workload(wl, img, precision="fp32k", device="cuda:0")
    print(f"[bench] lattice built: {lat.n} particles, {lat.m} springs", file=sys.stderr,
          flush=True)
    if args.workload == "c3":
        pass  # 3D: the gather kernel, one thread per particle
    elif args.autotune:
        lat.autotune(100)
    else:
        rows, pf = (int(v) for v in args.launch.split(","))
        lat.set_launch(args.kernel, rows)
        lat.set_prefetch(pf)
    launch = lat.launch()
    print(f"[bench] launch: {launch}", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        lat.apply_increment(wl["d_eps"])
        lat.relax(spi)
    lat.read_state()
    lat.set_timing(True)
    lat.read_timing()  # clear
    torch.cuda.synchronize()
    lat.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        lat.apply_increment(wl["d_eps"])
        lat.relax(spi)
        if (i + 1) % 50 == 0:
            print(f"[bench] {i + 1}/{args.steps} increments", file=sys.stderr, flush=True)
    lat.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rec = lat.read_state()
    kern_ms, kern_launches = lat.read_timing()
    lat.set_timing(False)

    springs = lat.m
    timesteps = args.steps * spi
    value = springs * timesteps / wall
    avg_step_s = kern_ms * 1e-3 / max(kern_launches, 1)  # event time per interior step
    spl = launch["steps_per_launch"]
    launch_s = avg_step_s * spl                            # per launch of the step kernel
    bytes_per_launch = lat.step_bytes()
    hbm_gbs = bytes_per_launch / launch_s / 1e9
    counters = measured_counters(launch) if args.workload == "c2" else None
    if args.workload == "c3":
        kname = "k_step<3,1,1> (fp32 compensated, one thread per particle)"
    else:
        kname = {2: "k_sweep2d_x2<1,1> (fp32 compensated, two interior steps per launch)",
                 1: "k_sweep2d<1,1,1,0> (fp32 compensated, one interior step per launch)"}[spl]
    roofline = {"bound": "hbm", "achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": hbm_gbs / HBM_PEAK_GBS,
                "traffic": counters.get("bytes_per_launch") if counters else None,
                "bytes_per_launch": bytes_per_launch, "steps_per_launch": spl, "kernel": kname}
    if counters and counters.get("valu_insts_per_launch"):
        # VALU issue rate: wavefront instructions x 64 lanes per launch time
        alu = counters["valu_insts_per_launch"] * 64 / launch_s / 1e12
        if alu / VALU_PEAK_T > roofline["frac"]:
            roofline.update({"bound": "alu", "achieved": alu, "peak": VALU_PEAK_T,
                             "unit": "T VALU lane-instructions/s", "frac": alu / VALU_PEAK_T,
                             "hbm_GBs": hbm_gbs, "hbm_frac": hbm_gbs / HBM_PEAK_GBS})
        else:
            roofline["alu_frac"] = alu / VALU_PEAK_T

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "spring-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD_NAMES[args.workload],
            "particles": lat.n,
            "springs": springs,
            "steps_per_increment": spi,
            "strain_at_end": rec["eps"],
            "broken_springs_at_end": rec["n_broken"],
            "step_kernel_us": avg_step_s * 1e6,
            "step_kernel_launch_us": launch_s * 1e6,
            "launch": launch,
            "hbm_fraction_of_wall": bytes_per_launch * timesteps / spl / wall / 1e9 / HBM_PEAK_GBS,
        },
        "roofline": roofline,
    }
    if args.copy_ref:
        # plain copy kernel of known size: reads and writes copy_ref MiB once
        n = args.copy_ref * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # one elementwise kernel: reads and writes MIB MiB
        torch.cuda.synchronize()
        out["copy_ref_mib"] = args.copy_ref
    if not args.no_batch:
        del lat
        torch.cuda.empty_cache()
        print("[bench] batched specimens", file=sys.stderr, flush=True)
        out["batched"] = batched_c4(args, torch, inputs, lsm)
        if not args.no_cpu:
            out["batched"]["cpu_baseline"] = cpu_c4(args, inputs)
    if args.workload == "c2" and not args.no_c1:
        print("[bench] c1 small lattice", file=sys.stderr, flush=True)
        out["c1"] = small_c1(args, inputs, lsm)
    if args.cnn_bench:
        print("[bench] surrogate network kernels", file=sys.stderr, flush=True)
        out["cnn"] = cnn_kernels(torch)
    if not args.no_surrogate and args.workload == "c2":
        print("[bench] surrogate pipeline", file=sys.stderr, flush=True)
        out["surrogate"] = surrogate_c5(args)
    if not args.no_cpu:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, img, args.cpu_steps if args.workload == "c2"
                                           else max(args.cpu_steps // 30, 2))
    print(json.dumps(out))


if __name__ == "__main__":
    main()

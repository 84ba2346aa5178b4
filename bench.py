"""Benchmark: spring-steps/s of the lattice spring model hot path on one GPU.

Headline workload: the 256^3 random-field voxel lattice (6,693,133
particles, 56,137,660 face + edge springs), FP64 displacements and forces
(the paper's arithmetic), displacement-controlled tension in increments of
0.05 % strain, 2000 damped velocity Verlet steps per increment.  One bench
"step" is one loading increment: strain increment + step-0 force
evaluation, 2000 step kernels (spring forces with critical-stretch
breaking, force accumulation, integration), end-of-increment reductions
and the break log.

spring-steps/s = springs in the list (broken ones included, they are still
iterated) x timesteps / wall time.  The roofline object rates the step
kernel by the per-timestep bytes of the explicit spring-list model,
B = N (2 s + 5) + 6 M (s: bytes of a particle's state, 48 in 3D FP64), over
its average duration per step measured with HIP events on the library's
stream; `traffic` is what rocprofv3 counted for the same kernel
(profiles/), or null when the kernel source differs from the one counted.

Further sections (each can be skipped): the same lattice in FP32 with
compensated displacements; the 2048^2 brick-and-mortar lattice in both
precisions over increments 41-80 (fracture and the stress peak); 4096
batched specimens to failure with the oracle on one and on all host cores;
the 32^2 lattice; the batched-model + surrogate pipeline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = ("spring-steps/s (% HBM roofline); specimens/hour batched+surrogate "
          "@≤5% error")
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-instructions/s
# (78.6 TFLOP/s of non-packed FP32 or FP64 FMA)
VALU_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12
KERNEL_SRC = os.path.join(ROOT, "paper_2201_04565_amd", "csrc", "lsm_kernels.hip")
COUNTERS = {"c3": os.path.join(ROOT, "profiles", "c3_step_counters.json"),
            "c2": os.path.join(ROOT, "profiles", "c2_step_counters.json")}
# bytes of a particle's state per step (read and written once each): 2D
# FP32-compensated (u_hi, u_lo, v) 24, FP64 32; 3D 36 / 48
STATE_BYTES = {(2, "fp32k"): 24, (2, "fp64"): 32, (3, "fp32k"): 36, (3, "fp64"): 48}
KERNEL_NAMES = {
    ("c3", "fp64"): "k_step_c3w<0, 2816, 0> (3D compact layout, neighbours staged in LDS windows, fp64)",
    ("c3", "fp32k"): "k_step_c3w<1, 2816, 0> (3D compact layout, neighbours staged in LDS windows, fp32 forces, compensated fp32 displacements)",
    ("c2", "fp32k"): "k_sweep2d_x2<1,1> (2D row sweep, two interior steps per launch, fp32 compensated)",
    ("c2", "fp64"): "k_sweep2d<0,1,1,0> (2D row sweep, fp64)",
}


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def host_cpu():
    """CPU model and logical core count of this host."""
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def survey_bytes(dim, precision, n, m):
    """Per-timestep bytes of the explicit spring-list model."""
    return n * (2 * STATE_BYTES[(dim, precision)] + 5) + 6 * m


def measured_counters(workload, precision, launch):
    """rocprofv3 counters of the step kernel (HBM bytes and VALU
    instructions per interior step) from the committed summary, or None when
    absent, taken on a different kernel source or another launch."""
    try:
        with open(COUNTERS[workload]) as f:
            t = json.load(f)
    except (OSError, ValueError, KeyError):
        return None
    t = t.get(precision) if isinstance(t, dict) else None
    if not t or t.get("kernel_src_sha256") != kernel_hash():
        return None
    want = {k: launch[k] for k in ("variant", "rows_per_wave", "prefetch")}
    if t.get("launch") != want:
        return None
    return t


def lattice_run(lsm, torch, wl, img, precision, warmup, timed, spi, workload, log):
    """Loading increments on one lattice: `warmup` untimed, `timed` timed
    (wall clock around them, HIP events around every interior-step chunk)."""
    lat = lsm.Lattice.from_workload(wl, img, precision=precision, device="cuda:0")
    launch = lat.launch()
    log(f"{workload} {precision}: {lat.n} particles, {lat.m} springs, launch {launch}")
    for i in range(warmup):
        lat.apply_increment(wl["d_eps"])
        lat.relax(spi)
        if (i + 1) % 20 == 0:
            log(f"  warm-up {i + 1}/{warmup}")
    lat.read_state()
    lat.set_timing(True)
    lat.read_timing()  # clear
    torch.cuda.synchronize()
    lat.synchronize()
    t0 = time.perf_counter()
    for i in range(timed):
        lat.apply_increment(wl["d_eps"])
        lat.relax(spi)
        if (i + 1) % 20 == 0:
            log(f"  timed {i + 1}/{timed}")
    lat.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rec0 = lat.read_state()
    kern_ms, kern_steps = lat.read_timing()
    lat.set_timing(False)
    dim = 3 if img.ndim == 3 else 2
    step_s = kern_ms * 1e-3 / max(kern_steps, 1)   # events per interior step
    B = survey_bytes(dim, precision, lat.n, lat.m)
    spl = launch["steps_per_launch"]
    implicit = lat.step_bytes() / spl               # this layout's own bytes per step
    counters = measured_counters(workload, precision, launch)
    roof = {"bound": "hbm", "achieved": B / step_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": B / step_s / 1e9 / HBM_PEAK_GBS,
            "traffic": counters["bytes_per_step"] if counters else None,
            "bytes_per_step": B, "bytes_model": "N(2s+5)+6M per timestep, s=%d" % STATE_BYTES[(dim, precision)],
            "implicit_bytes_per_step": implicit,
            "implicit_frac": implicit / step_s / 1e9 / HBM_PEAK_GBS,
            "kernel": KERNEL_NAMES.get((workload, precision), launch["variant"])}
    if counters:
        roof["traffic_GBs"] = counters["bytes_per_step"] / step_s / 1e9
        if counters.get("valu_insts_per_step"):
            # VALU issue rate: wavefront instructions x 64 lanes per step time
            roof["valu_frac"] = counters["valu_insts_per_step"] * 64 / step_s / 1e12 / VALU_PEAK_T
    out = dict(value=lat.m * timed * spi / wall, unit="spring-steps/s", ms_per_increment=wall * 1e3 / timed,
               particles=lat.n, springs=lat.m, steps_per_increment=spi, increments_timed=timed,
               increments_before=warmup, strain_at_end=rec0["eps"], broken_springs_at_end=rec0["n_broken"],
               step_kernel_us=step_s * 1e6, launch=launch, roofline=roof)
    del lat
    torch.cuda.empty_cache()
    return out


def extensions(torch, inputs, lsm, log):
    """The paper's protocol, local fields and the spring laws, each timed on
    a full-size lattice: constant strain-rate loading of the C2 bricks
    (grips moved before every step, one interior step per launch), the local
    stress and strain fields of the C3 lattice, and the cubic spring law on
    C3 (gather kernel).  HIP events on the library's stream."""
    import ctypes as C

    out = {}
    # f1: grips at a constant strain rate, a record every 500 steps
    w2 = inputs.WORKLOADS["c2"]
    lat = lsm.Lattice.from_workload(w2, inputs.c2_image(), precision="fp32k", device="cuda:0")
    lat.relax_trace(1e-6, 100, 100)  # graphs captured, grips running
    lat.set_timing(True)
    lat.read_timing()
    t0 = time.perf_counter()
    recs = lat.relax_trace(1e-6, 2000, 500)
    wall = time.perf_counter() - t0
    ms, steps = lat.read_timing()
    lat.set_timing(False)
    step_s = ms * 1e-3 / max(steps, 1)
    B = survey_bytes(2, "fp32k", lat.n, lat.m)
    own = lat.step_bytes() / lat.launch()["steps_per_launch"]
    out["rate"] = dict(workload="c2 bricks 2048^2, fp32 compensated, strain rate 1e-6 per unit time, "
                                "2000 steps, a record every 500",
                       launch=lat.launch(), us_per_step=step_s * 1e6, spring_steps_per_s=lat.m / step_s,
                       wall_s=wall, records=len(recs), strain_at_end=recs[-1]["eps"],
                       roofline={"bound": "hbm", "achieved": B / step_s / 1e9, "peak": HBM_PEAK_GBS,
                                 "unit": "GB/s", "frac": B / step_s / 1e9 / HBM_PEAK_GBS,
                                 "bytes_per_step": B, "implicit_bytes_per_step": own,
                                 "implicit_frac": own / step_s / 1e9 / HBM_PEAK_GBS})
    log(f"rate: {out['rate']['us_per_step']:.1f} us per step")
    del lat
    torch.cuda.empty_cache()
    # f2: local fields of the C3 lattice after one increment
    w3 = inputs.WORKLOADS["c3"]
    img3 = inputs.c3_image()
    lat = lsm.Lattice.from_workload(w3, img3, precision="fp64", device="cuda:0")
    lat.apply_increment(w3["d_eps"])
    lat.relax(200)
    lat.read_state()
    n = lat.n
    stress = torch.empty(n * 9, dtype=torch.float64, device="cuda:0")
    strain = torch.empty(n * 9, dtype=torch.float64, device="cuda:0")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fields = {}
    for radius in (0, 1):
        for rep_ in range(2):  # the second pass is timed
            e0.record(lat.stream)
            for _ in range(5):
                lat._check(lat._L.lsm_local_fields(lat._h, radius, C.c_void_p(stress.data_ptr()),
                                                   C.c_void_p(strain.data_ptr())))
            e1.record(lat.stream)
            e1.synchronize()
        t = e0.elapsed_time(e1) / 5 * 1e-3
        # state read once (u, v 24 B each, mask 4, flag 1, site index 4), the
        # per-particle virial written and read once (72 B each), stress and
        # strain written once (72 B each)
        fb = n * (24 + 24 + 4 + 1 + 4 + 72 + 72 + 72 + 72)
        fields[f"radius{radius}"] = dict(ms_per_call=t * 1e3, particles_per_s=n / t,
                                         roofline={"bound": "hbm", "achieved": fb / t / 1e9, "peak": HBM_PEAK_GBS,
                                                   "unit": "GB/s", "frac": fb / t / 1e9 / HBM_PEAK_GBS,
                                                   "bytes_per_call": fb})
    out["fields"] = dict(workload="c3 random-field voxels 256^3, fp64, local virial stress over the radius-0 / "
                                  "radius-1 domain and Lagrangian strain of every particle", particles=n, **fields)
    log(f"fields: {fields['radius1']['ms_per_call']:.2f} ms per call (radius 1)")
    del lat, stress, strain
    torch.cuda.empty_cache()
    # f3: the cubic spring law (the gather kernel)
    lat = lsm.Lattice.from_workload(w3, img3, precision="fp64", device="cuda:0", spring_law="cubic", law_c=1.0)
    lat.apply_increment(w3["d_eps"])
    lat.relax(200)
    lat.read_state()
    lat.set_timing(True)
    lat.read_timing()
    lat.relax(1000)
    ms, steps = lat.read_timing()
    lat.set_timing(False)
    step_s = ms * 1e-3 / max(steps, 1)
    B = survey_bytes(3, "fp64", lat.n, lat.m)
    out["cubic_law"] = dict(workload="c3 random-field voxels 256^3, fp64, cubic spring law (c = 1), 1000 steps",
                            launch=lat.launch(), us_per_step=step_s * 1e6, spring_steps_per_s=lat.m / step_s,
                            roofline={"bound": "hbm", "achieved": B / step_s / 1e9, "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": B / step_s / 1e9 / HBM_PEAK_GBS,
                                      "bytes_per_step": B})
    log(f"cubic law: {out['cubic_law']['us_per_step']:.1f} us per step")
    del lat
    torch.cuda.empty_cache()
    return out


def cpu_baseline(wl, img, steps: int):
    """The FP64 oracle, single thread, on part of one increment of the same
    lattice (per-step cost does not change along the run)."""
    import oracle
    prm = oracle.Params(k=wl["k"], s=wl["s"], mass=wl["mass"], a=wl.get("a", 1.0),
                        k_face=wl.get("k_face", 1.0), k_diag=wl.get("k_diag", 1.0),
                        dt=wl["dt"], gamma=wl["gamma"], void_value=wl.get("void_value", -1))
    net = oracle.Net.lattice(img, prm)
    t0 = time.perf_counter()
    net.apply_increment(wl["d_eps"])
    net.relax(steps)
    dt = time.perf_counter() - t0
    model, ncpu = host_cpu()
    return dict(value=net.m * steps / dt, unit="spring-steps/s", cores=1, kind="oracle",
                sample=f"full {'x'.join(str(d) for d in img.shape[::-1])} lattice, 1 increment, "
                       f"{steps} steps (+ step-0 evaluation), FP64, single thread, {dt:.1f} s",
                cpu_model=model, host_logical_cpus=ncpu)


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


def _oracle_specimen(task):
    """One specimen through `inc` increments on the oracle (one process)."""
    import oracle
    from paper_2201_04565_amd import inputs
    seed, inc = task
    wl = inputs.WORKLOADS["c4"]
    img = inputs.batch_specimens(1, seed0=seed)[0]
    net = oracle.Net.lattice(img, oracle.Params(k=wl["k"], s=wl["s"], mass=wl["mass"], dt=wl["dt"],
                                                gamma=wl["gamma"]))
    t0 = time.perf_counter()
    for _ in range(inc):
        net.apply_increment(wl["d_eps"])
        net.relax(wl["steps"])
    return img.shape[0], time.perf_counter() - t0


def cpu_c4(args, inputs, pool):
    """The oracle on the host: one core (one specimen per side for a prefix
    of increments, extrapolated to the batch's increments; per-step cost is
    constant because broken springs stay in the list) and all cores (one
    specimen per core, the first specimens of the batch, run together in
    `pool`, worker processes started before the GPU was touched)."""
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
    model, ncpu = host_cpu()
    out = dict(value=len(imgs) / total * 3600.0, unit="specimens/hour", cores=1, kind="oracle",
               sample=f"one specimen per side, {args.cpu_c4_inc} increments each, "
                      f"extrapolated to {wl['max_inc']} increments per specimen",
               cpu_model=model, host_logical_cpus=ncpu)
    # all cores: specimens of the batch spread over the worker processes; the
    # single-core time of the same work over the wall time is the speedup
    # the host's cores give, applied to the single-core rate
    P = pool._processes
    tasks = [(1000 + i, args.cpu_c4_inc) for i in range(3 * P)]
    t0 = time.perf_counter()
    res = pool.map(_oracle_specimen, tasks, chunksize=1)
    wall = time.perf_counter() - t0
    single = sum(per_step.get(int(L), float(np.mean(list(per_step.values())))) * args.cpu_c4_inc * wl["steps"]
                 for L, _ in res)
    speedup = single / wall
    out["all_cores"] = dict(value=out["value"] * speedup, unit="specimens/hour", cores=P, kind="oracle",
                            speedup_over_one_core=speedup,
                            sample=f"{len(tasks)} specimens of the batch (seeds 1000-{999 + len(tasks)}) over "
                                   f"{P} processes, {args.cpu_c4_inc} increments each, {wall:.1f} s wall")
    return out


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
    labels from the batched model, a 5-member ensemble trained on them, a
    spread gate calibrated on a validation split (at most 5 %, accepted
    95th-percentile modulus error within 5 % there) with fallback to the
    model; specimens/hour of the pipeline and of the batched model alone,
    the modulus error against the model's own labels, and the cost
    including the labelling and training that built the surrogate."""
    from paper_2201_04565_amd import surrogate as S

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    img_tr = S.specimen_images(args.sur_train, 10 ** 6)
    img_va = S.specimen_images(args.sur_val, 3 * 10 ** 6)
    img_te = S.specimen_images(args.sur_test, 2 * 10 ** 6)
    log(f"images generated ({time.perf_counter() - t0:.1f} s)")
    lab_tr = S.label(img_tr, log=log)
    lab_va = S.label(img_va, log=log)
    lab_te = S.label(img_te, log=log)
    sur = S.Surrogate(k=5, batch=512, seed=0)
    sur.fit(img_tr, S.targets(lab_tr), epochs=args.sur_epochs, lr=2e-3, log=log)
    cal = S.calibrate_gate(sur, img_va, lab_va, target_p95=0.05, max_gate=0.05)
    res = S.evaluate(sur, img_te, lab_te, gate=cal["gate"])
    model_per = lab_te.seconds / len(img_te)
    res.update(
        workload=f"{args.sur_train} train / {args.sur_val} validation / {args.sur_test} test 128x128 "
                 f"inclusion specimens, labels = 64-point sigma_xx curve + modulus (64 x 0.5% x 500 steps, "
                 f"fp32), 5-member BF16 CNN ensemble, {args.sur_epochs} epochs, gate calibrated on the "
                 f"validation split",
        calibration=cal,
        label_specimens_per_hour=len(img_tr) / lab_tr.seconds * 3600.0,
        batched_model_specimens_per_hour=len(img_te) / lab_te.seconds * 3600.0,
        train_s=sur.train_seconds,
        train_TFLOPs=3 * cnn_forward_flops() * 5 * args.sur_epochs * (len(img_tr) // 512) * 512
        / sur.train_seconds / 1e12,
        amortized=S.amortized(res, lab_tr.seconds + lab_va.seconds, sur.train_seconds, model_per),
        total_s=time.perf_counter() - t0)
    res["pipeline_over_batched_model"] = res["specimens_per_hour"] / res["batched_model_specimens_per_hour"]
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("c3", "c2"), default="c3",
                    help="headline lattice: c3 256^3 random-field voxels (default), c2 2048^2 bricks")
    ap.add_argument("--dtype", choices=("f64", "f32k"), default="f64",
                    help="headline arithmetic: f64 (the paper's, default) or fp32 forces with "
                         "compensated fp32 displacements")
    ap.add_argument("--steps", type=int, default=10, help="timed loading increments of the headline")
    ap.add_argument("--warmup", type=int, default=2, help="untimed loading increments before them")
    ap.add_argument("--steps-per-inc", type=int, default=None)
    ap.add_argument("--cpu-steps", type=int, default=30, help="oracle timesteps of the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only-headline", action="store_true", help="skip every further section")
    ap.add_argument("--no-c3-fp32k", action="store_true")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--c2-from", type=int, default=40, help="c2 section: increments before the timed ones")
    ap.add_argument("--c2-steps", type=int, default=40, help="c2 section: timed increments")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched C4 measurement")
    ap.add_argument("--batch-n", type=int, default=4096)
    ap.add_argument("--plain-per-size", type=int, default=2)
    ap.add_argument("--cpu-c4-inc", type=int, default=1)
    ap.add_argument("--cpu-workers", type=int, default=16, help="processes of the all-core oracle run")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--cnn-bench", action="store_true", help="also time the surrogate network kernels")
    ap.add_argument("--no-c1", action="store_true", help="skip the small-lattice (C1) section")
    ap.add_argument("--no-ext", action="store_true",
                    help="skip the strain-rate, local-field and spring-law section")
    ap.add_argument("--sur-train", type=int, default=4096,
                    help="training specimens (the full C5 configuration: 50000)")
    ap.add_argument("--sur-val", type=int, default=1024, help="validation specimens (C5: 5000)")
    ap.add_argument("--sur-test", type=int, default=1024, help="test specimens (C5: 5000)")
    ap.add_argument("--sur-epochs", type=int, default=20, help="epochs (as C5)")
    ap.add_argument("--copy-ref", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (counter scale reference)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (a single "
              "lattice would shard as x-slabs with a halo exchange, a batch by specimen)",
              file=sys.stderr)
        sys.exit(2)
    if args.only_headline:
        args.no_c3_fp32k = args.no_c2 = args.no_batch = args.no_c1 = args.no_surrogate = args.no_ext = True
    pool = None
    if not args.no_batch and not args.no_cpu:
        # the all-core oracle workers start now, before anything touches the
        # GPU, and wait idle until the GPU sections are done
        import multiprocessing as mp
        pool = mp.get_context("spawn").Pool(max(1, min(args.cpu_workers, os.cpu_count() or 1)))

    import torch

    from paper_2201_04565_amd import inputs, lsm

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    prec = "fp64" if args.dtype == "f64" else "fp32k"
    wl = inputs.WORKLOADS[args.workload]
    spi = args.steps_per_inc or wl["steps"]
    img = inputs.c3_image() if args.workload == "c3" else inputs.c2_image()
    head = lattice_run(lsm, torch, wl, img, prec, args.warmup, args.steps, spi, args.workload, log)
    names = {"c3": "c3 256^3 simple-cubic voxel lattice from a thresholded Gaussian random field (40% solid, "
                   "largest cluster), face + edge springs, 0.05% strain increments x 2000 steps",
             "c2": "c2 brick-and-mortar 2048x2048 triangular lattice, 0.05% strain increments x 2000 steps"}
    arith = {"fp64": "fp64 positions and forces", "fp32k": "fp32 forces, compensated fp32 displacements"}
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "spring-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_increment"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{names[args.workload]}, {arith[prec]}",
            **{k: head[k] for k in ("particles", "springs", "steps_per_increment", "strain_at_end",
                                    "broken_springs_at_end", "step_kernel_us", "launch")},
        },
        "roofline": head["roofline"],
    }
    if args.copy_ref:
        # plain copy kernel of known size: reads and writes copy_ref MiB once
        n = args.copy_ref * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        out["copy_ref_mib"] = args.copy_ref
        del src, dst
    if args.workload == "c3" and prec == "fp64" and not args.no_c3_fp32k:
        out["c3_fp32k"] = lattice_run(lsm, torch, wl, img, "fp32k", args.warmup, args.steps, spi, "c3", log)
    if not args.no_c2:
        w2 = inputs.WORKLOADS["c2"]
        img2 = inputs.c2_image()
        out["c2"] = {"workload": names["c2"] + f", increments {args.c2_from + 1}-{args.c2_from + args.c2_steps}",
                     "mall_caveat": "the state fits the 256 MB Infinity Cache, so the HBM fraction may count "
                                    "cache-served bytes"}
        for p2 in ("fp32k", "fp64"):
            out["c2"][p2] = lattice_run(lsm, torch, w2, img2, p2, args.c2_from, args.c2_steps, w2["steps"],
                                        "c2", log)
    if not args.no_batch:
        log("batched specimens")
        out["batched"] = batched_c4(args, torch, inputs, lsm)
        if not args.no_cpu:
            out["batched"]["cpu_baseline"] = cpu_c4(args, inputs, pool)
    if not args.no_c1:
        log("c1 small lattice")
        out["c1"] = small_c1(args, inputs, lsm)
    if not args.no_ext:
        log("strain-rate loading, local fields, cubic spring law")
        out["extensions"] = extensions(torch, inputs, lsm, log)
    if args.cnn_bench:
        log("surrogate network kernels")
        out["cnn"] = cnn_kernels(torch)
    if not args.no_surrogate:
        log("surrogate pipeline")
        out["surrogate"] = surrogate_c5(args)
    if not args.no_cpu:
        log("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(wl, img, args.cpu_steps)
    if pool is not None:
        pool.close()
        pool.join()
    print(json.dumps(out))


if __name__ == "__main__":
    main()

"""Seeded synthetic phase images for the lattice spring model workloads.

This module only draws images (numpy arrays of uint8 phase labels); it holds
none of the method's arithmetic, so both the CPU oracle and the GPU path can
consume its output.  Every generator is deterministic given its seed
(``numpy.random.default_rng``, PCG64).

Image convention: 2D images have shape ``(ny, nx)``, 3D images ``(nz, ny, nx)``;
x is the fastest axis and row 0 is ``y = 0``.  The pixel value is the phase
index (0 .. nphase-1); ``VOID`` marks an empty site.

The paper builds its specimens from images with a gray-scale-to-type mapping
(Introduction) and tests Poisson composites with soft inclusions (Section 3.1);
its own input files are not available, so these generators stand in for them.
"""
from __future__ import annotations

import numpy as np

VOID = 255

# Phase labels used by the two-phase workloads.
SOFT = 0
STIFF = 1


def bernoulli_two_phase(nx: int = 32, ny: int = 32, p_stiff: float = 0.3,
                        seed: int = 0) -> np.ndarray:
    """Each pixel is STIFF with probability ``p_stiff``, else SOFT."""
    rng = np.random.default_rng(seed)
    u = rng.random((ny, nx))
    return np.where(u < p_stiff, STIFF, SOFT).astype(np.uint8)


def brick_and_mortar(nx: int = 2048, ny: int = 2048, brick_w: int = 32,
                     brick_h: int = 8, mortar: int = 2, jitter: float = 0.2,
                     seed: int = 1) -> np.ndarray:
    """Running-bond brick wall: STIFF bricks in a SOFT mortar.

    Brick rows have pitch ``brick_h + mortar``; within a row the bricks have
    pitch ``brick_w + mortar``.  Row ``r`` is offset by half a pitch on odd
    rows plus a seeded jitter uniform in ``(-jitter, jitter) * brick_w``
    pixels, rounded to an integer.
    """
    rng = np.random.default_rng(seed)
    px = brick_w + mortar
    py = brick_h + mortar
    nrows = (ny + py - 1) // py
    offs = ((np.arange(nrows) % 2) * (px // 2)
            + np.rint(rng.uniform(-jitter, jitter, nrows) * brick_w)).astype(np.int64)
    img = np.full((ny, nx), SOFT, dtype=np.uint8)
    x = np.arange(nx, dtype=np.int64)
    for r in range(nrows):
        y0 = r * py
        y1 = min(y0 + brick_h, ny)
        if y0 >= ny:
            break
        in_brick = np.mod(x - offs[r], px) < brick_w
        img[y0:y1, in_brick] = STIFF
    return img


def _largest_cluster_18(solid: np.ndarray) -> np.ndarray:
    """Keep the largest solid cluster under 18-connectivity (face + edge)."""
    from scipy import ndimage
    struct = ndimage.generate_binary_structure(3, 2)  # 18-neighbourhood
    lab, nlab = ndimage.label(solid, structure=struct)
    if nlab == 0:
        return solid
    sizes = np.bincount(lab.ravel())
    sizes[0] = 0
    return lab == int(np.argmax(sizes))


def gaussian_random_field_3d(n: int = 256, corr_len: float = 8.0,
                             solid_fraction: float = 0.4, seed: int = 2,
                             keep_largest: bool = True) -> np.ndarray:
    """Thresholded periodic Gaussian random field on an ``n^3`` voxel grid.

    White noise is filtered in Fourier space with a Gaussian of standard
    deviation ``corr_len / sqrt(2)`` (so the field covariance is
    ``exp(-r^2 / (2 corr_len^2))``), thresholded at the quantile that makes
    ``solid_fraction`` of the voxels solid, and reduced to its largest
    18-connected solid cluster.  Solid voxels get phase 0, the rest VOID.
    """
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((n, n, n)).astype(np.float64)
    k = np.fft.fftfreq(n) * 2.0 * np.pi
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    s = corr_len / np.sqrt(2.0)
    filt = np.exp(-0.5 * (kx * kx + ky * ky + kz * kz) * s * s)
    field = np.fft.ifftn(np.fft.fftn(noise) * filt).real
    thr = np.quantile(field, 1.0 - solid_fraction)
    solid = field > thr
    if keep_largest:
        solid = _largest_cluster_18(solid)
    img = np.full((n, n, n), VOID, dtype=np.uint8)
    img[solid] = 0
    return img


def circular_inclusions(L: int, seed: int, r_min: float = 3.0, r_max: float = 12.0,
                        vf_min: float = 0.1, vf_max: float = 0.4) -> np.ndarray:
    """STIFF matrix with SOFT circular inclusions placed as a Poisson process.

    A target area fraction is drawn uniformly in ``[vf_min, vf_max]``; disks of
    radius uniform in ``[r_min, r_max]`` with uniformly distributed centres
    (overlaps allowed) are added until the soft fraction reaches the target.
    """
    rng = np.random.default_rng(seed)
    target = rng.uniform(vf_min, vf_max)
    img = np.full((L, L), STIFF, dtype=np.uint8)
    yy, xx = np.mgrid[0:L, 0:L]
    soft = np.zeros((L, L), dtype=bool)
    n_soft = 0
    goal = target * L * L
    while n_soft < goal:
        r = rng.uniform(r_min, r_max)
        cx = rng.uniform(0, L)
        cy = rng.uniform(0, L)
        x0, x1 = max(int(cx - r) - 1, 0), min(int(cx + r) + 2, L)
        y0, y1 = max(int(cy - r) - 1, 0), min(int(cy + r) + 2, L)
        sub = (xx[y0:y1, x0:x1] + 0.5 - cx) ** 2 + (yy[y0:y1, x0:x1] + 0.5 - cy) ** 2 <= r * r
        soft[y0:y1, x0:x1] |= sub
        n_soft = int(soft.sum())
    img[soft] = SOFT
    return img


def edge_notch(img: np.ndarray, depth: int, width: int = 1, x0: int | None = None) -> np.ndarray:
    """Copy of a 2D image with a straight notch of VOID pixels for a mode-I
    test under tension along x: ``width`` columns starting at ``x0`` (default:
    centred), from the bottom edge (row 0) up to row ``depth - 1``.  The
    paper's specimens carry such a notch (Section 3.1 mode-I tests; its size
    is only drawn in a figure, so it is a parameter here)."""
    out = np.array(img, dtype=np.uint8, copy=True)
    ny, nx = out.shape
    if x0 is None:
        x0 = (nx - width) // 2
    out[:max(0, min(depth, ny)), max(0, x0):min(nx, x0 + width)] = VOID
    return out


def notched_composite(L: int = 96, seed: int = 7, depth_frac: float = 0.2) -> np.ndarray:
    """A Poisson composite (STIFF matrix, SOFT inclusions placed as a Poisson
    process, Section 3.1) of side ``L`` with a centred one-pixel edge notch
    of depth ``depth_frac * L``."""
    return edge_notch(circular_inclusions(L, seed=seed), int(round(depth_frac * L)))


def uniform_phase(L: int, phase: int = SOFT) -> np.ndarray:
    """A single-phase square image (e.g. all soft)."""
    return np.full((L, L), phase, dtype=np.uint8)


def checkerboard(L: int, cell: int = 1) -> np.ndarray:
    """STIFF and SOFT squares of side ``cell`` alternating in x and y."""
    yy, xx = np.mgrid[0:L, 0:L]
    return np.where(((xx // cell) + (yy // cell)) % 2 == 0, STIFF, SOFT).astype(np.uint8)


BATCH_SIZES = (64, 96, 128, 192, 256)


def batch_specimens(n: int = 4096, seed0: int = 1000, sizes=BATCH_SIZES):
    """Specimen ``i`` uses seed ``seed0 + i``: its size is drawn from ``sizes``
    and its image from :func:`circular_inclusions`."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(seed0 + i)
        L = int(sizes[int(rng.integers(0, len(sizes)))])
        out.append(circular_inclusions(L, seed=seed0 + i))
    return out


def perturbation(n: int, dim: int, scale: float, seed: int) -> np.ndarray:
    """Seeded uniform position perturbations in ``[-scale, scale]``."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=(n, dim))


# ---------------------------------------------------------------------------
# Workload definitions (numbers only).  Phase labels: SOFT = 0, STIFF = 1 for
# the two-phase images; the single solid phase of the 3D field is 0.  Off-
# diagonal NaN entries select the series rule for interface springs.
NAN = float("nan")

WORKLOADS = {
    # 32x32 Bernoulli(0.3) two-phase image, FP64, 20 increments of 0.5 %.
    "c1": dict(dim=2, k=[[0.1, NAN], [NAN, 1.0]], s=[[0.20, NAN], [NAN, 0.05]],
               mass=[1.0, 1.0], a=1.0, dt=0.01, gamma=0.1, d_eps=0.005, n_inc=20,
               steps=500, precision="fp64", void_value=-1),
    # 2048x2048 brick-and-mortar, FP32 forces with compensated displacements.
    "c2": dict(dim=2, k=[[0.05, NAN], [NAN, 1.0]], s=[[0.30, NAN], [NAN, 0.02]],
               mass=[1.0, 1.0], a=1.0, dt=0.01, gamma=0.1, d_eps=0.0005, n_inc=200,
               steps=2000, precision="fp32k", void_value=-1),
    # 256^3 Gaussian-random-field solid (40 %), face + edge springs.
    "c3": dict(dim=3, k=[[1.0]], s=[[0.03]], mass=[1.0], a=1.0, k_face=1.0, k_diag=0.5,
               dt=0.01, gamma=0.1, d_eps=0.0005, n_inc=100, steps=2000,
               precision="fp32k", void_value=VOID),
    # the paper's own loading of a notched Poisson composite (Section 3.1):
    # spring constants and critical lengths of its spring table (stiff-stiff
    # 2e-3 / 10.1, soft-soft 2e-5 / 11.0, stiff-soft 1.25e-4 / 10.4 at r0 = 10,
    # as critical stretches), unit masses, dt = 1, no damping, grips pulled
    # apart at a strain rate of 1e-6 per unit time, energies every 500 steps.
    "mode1": dict(dim=2, k=[[2.0e-5, 1.25e-4], [1.25e-4, 2.0e-3]],
                  s=[[0.10, 0.04], [0.04, 0.01]], mass=[1.0, 1.0], a=10.0, dt=1.0,
                  gamma=0.0, rate=1e-6, steps=16000, every=500, precision="fp64",
                  void_value=VOID),
    # batched circular-inclusion specimens: stiff matrix, soft inclusions.
    "c4": dict(dim=2, k=[[0.1, NAN], [NAN, 1.0]], s=[[0.20, NAN], [NAN, 0.05]],
               mass=[1.0, 1.0], a=1.0, dt=0.01, gamma=0.1, d_eps=0.005, max_inc=64,
               steps=500, precision="fp32k", void_value=-1),
}


def c1_image():
    return bernoulli_two_phase(32, 32, 0.3, seed=0)


def c2_image(n: int = 2048):
    return brick_and_mortar(n, n, seed=1)


def c3_image(n: int = 256):
    return gaussian_random_field_3d(n, seed=2)

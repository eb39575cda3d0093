"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module holds no arithmetic of the reconstruction method itself: it only
draws random numbers (phantoms, noise, the Gaussian test matrix Omega, power
iteration start vectors), samples point-spread functions and rounds arrays to
storage precisions.  Measurements y = A x + noise are formed by whichever side
consumes these inputs, with its own operator.

The synthetic workloads stand in for the paper's natural test images, the AAPM
CT slices and the walnut data (Sec. IV), none of which is available; they keep
the shapes, value ranges and noise models the five benchmark workloads name.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = [
    "rng", "gaussian_psf", "phantom_blocks", "phantom_ellipses", "omega",
    "gaussian", "salt_pepper_masks", "round_bf16", "round_dtype",
    "Workload", "WORKLOADS", "workload", "BatchInstance", "batch_instances",
]


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    """PCG64 generator for (seed, stream); streams keep draws independent."""
    return np.random.Generator(np.random.PCG64([int(seed), int(stream)]))


def gaussian_psf(k: int, sigma: float) -> np.ndarray:
    """k x k Gaussian point-spread function, centred at (k-1)/2, sum 1.

    Sampled at integer offsets and truncated to the k x k support (Sec. IV-A
    names only the size and the standard deviation).
    """
    if k < 1 or k % 2 == 0:
        raise ValueError("PSF size must be odd and positive")
    c = (k - 1) / 2.0
    a = np.arange(k, dtype=np.float64) - c
    h = np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / (2.0 * sigma * sigma))
    return h / h.sum()


def phantom_blocks(n: int, seed: int, n_ellipses: int = 8,
                   n_rects: int = 4) -> np.ndarray:
    """Piecewise-constant n x n phantom in [0, 1].

    Painter's overwrite on a zero background: ellipses first, then
    axis-aligned rectangles, each with a value drawn from U[0, 1].
    """
    g = rng(seed, 1)
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    xx = (xx + 0.5) / n - 0.5
    yy = (yy + 0.5) / n - 0.5
    img = np.zeros((n, n))
    for _ in range(n_ellipses):
        cx, cy = g.uniform(-0.35, 0.35, 2)
        ax, ay = g.uniform(0.05, 0.3, 2)
        th = g.uniform(0, np.pi)
        val = g.uniform(0, 1)
        xr = (xx - cx) * np.cos(th) + (yy - cy) * np.sin(th)
        yr = -(xx - cx) * np.sin(th) + (yy - cy) * np.cos(th)
        img[(xr / ax) ** 2 + (yr / ay) ** 2 <= 1.0] = val
    for _ in range(n_rects):
        cx, cy = g.uniform(-0.4, 0.4, 2)
        hx, hy = g.uniform(0.03, 0.2, 2)
        val = g.uniform(0, 1)
        img[(np.abs(xx - cx) <= hx) & (np.abs(yy - cy) <= hy)] = val
    return img


def phantom_ellipses(n: int, seed: int, n_ellipses: int = 12,
                     vmax: float = 0.04) -> np.ndarray:
    """CT phantom: ellipses inside the inscribed disc, values U[0, vmax]."""
    g = rng(seed, 2)
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    xx = (xx + 0.5) / n - 0.5
    yy = (yy + 0.5) / n - 0.5
    img = np.zeros((n, n))
    # a body ellipse first so most of the disc carries attenuation
    body = (xx / 0.42) ** 2 + (yy / 0.36) ** 2 <= 1.0
    img[body] = g.uniform(0.5, 0.8) * vmax
    for _ in range(n_ellipses - 1):
        r = g.uniform(0, 0.3)
        phi = g.uniform(0, 2 * np.pi)
        cx, cy = r * np.cos(phi), r * np.sin(phi)
        ax, ay = g.uniform(0.02, 0.12, 2)
        th = g.uniform(0, np.pi)
        xr = (xx - cx) * np.cos(th) + (yy - cy) * np.sin(th)
        yr = -(xx - cx) * np.sin(th) + (yy - cy) * np.cos(th)
        img[(xr / ax) ** 2 + (yr / ay) ** 2 <= 1.0] = g.uniform(0, vmax)
    img[xx ** 2 + yy ** 2 > 0.25] = 0.0
    return img


def omega(ell: int, n1: int, n2: int, seed: int) -> np.ndarray:
    """Gaussian test matrix, stored as ell images of n1 x n2 (Alg. 1, step 1)."""
    return rng(seed, 3).standard_normal((ell, n1, n2))


def gaussian(shape, seed: int, stream: int = 4) -> np.ndarray:
    """Standard normal array (measurement noise, power-iteration starts)."""
    return rng(seed, stream).standard_normal(shape)


def salt_pepper_masks(shape, seed: int, frac: float = 0.05):
    """Two disjoint index masks: `frac` of the entries set to 1, then another
    `frac` of the remaining ones set to 0 (Sec. IV-A footnote)."""
    g = rng(seed, 5)
    m = int(np.prod(shape))
    perm = g.permutation(m)
    k = int(round(frac * m))
    salt = np.zeros(m, bool)
    pepper = np.zeros(m, bool)
    salt[perm[:k]] = True
    pepper[perm[k:2 * k]] = True
    return salt.reshape(shape), pepper.reshape(shape)


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round float64 values to bfloat16 (nearest, ties to even); float64 out."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_dtype(a: np.ndarray, dtype: str) -> np.ndarray:
    """Round to the storage dtype ('f64', 'f32', 'bf16'); returns float64."""
    if dtype == "f64":
        return np.asarray(a, np.float64)
    if dtype == "f32":
        return np.asarray(a, np.float32).astype(np.float64)
    if dtype == "bf16":
        return round_bf16(a)
    raise ValueError(dtype)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One benchmark workload; sizes and parameters only."""
    name: str
    op: str                 # 'blur' | 'blurdown' | 'ct' | 'fan'
    n: int                  # image side (high resolution for 'blurdown')
    reg: str                # 'tv' | 'hs1' | 'l1haar3'
    lam: float
    ell: int
    dtype: str              # solver dtype: 'f64' | 'f32'
    sketch_dtype: str       # 'f64' | 'f32' | 'bf16'
    psf_k: int = 0
    psf_sigma: float = 0.0
    factor: int = 1
    views: int = 0
    bins: int = 0
    noise_sigma: float = 0.0
    noise_rel_max: float = 0.0
    salt_pepper: float = 0.0
    loss: str = "ls"        # 'ls' | 'huber'
    huber_delta: float = 0.0
    outer: int = 100
    inner: int = 20
    count: int = 1          # instances (the batched workload)
    smooth_eps: float = 0.0 # |r| -> sqrt(r^2 + eps) in the IRM weights
    fan: tuple = (0.0, 0.0, 1.0)   # 'fan': source radius, detector radius, bin spacing (pixels)

    @property
    def m_shape(self):
        if self.op == "blur":
            return (self.n, self.n)
        if self.op == "blurdown":
            return (self.n // self.factor, self.n // self.factor)
        return (self.views, self.bins)


WORKLOADS = {
    # 128^2 deblur, FP64, isotropic TV, ell = 32, 100 outer x 20 inner.
    "deblur128_tv_f64": Workload(
        "deblur128_tv_f64", "blur", 128, "tv", 1e-3, 32, "f64", "f64",
        psf_k=9, psf_sigma=1.5, noise_sigma=0.01, outer=100, inner=20),
    # 512^2 -> 256^2 super-resolution, Huber + Haar-3 l1, BF16 sketch.
    "sr512_haar_bf16": Workload(
        "sr512_haar_bf16", "blurdown", 512, "l1haar3", 5e-3, 64, "f32",
        "bf16", psf_k=7, psf_sigma=1.2, factor=2, noise_sigma=0.005,
        salt_pepper=0.05, loss="huber", huber_delta=0.01, outer=100),
    # 512^2 parallel-beam CT, 720 views x 736 bins, HS1, ell = 100.
    "ct512_hs1_f32": Workload(
        "ct512_hs1_f32", "ct", 512, "hs1", 2e-4, 100, "f32", "f32",
        views=720, bins=736, noise_rel_max=0.01, outer=200, inner=20),
    # 512^2 fan-beam CT as in the paper's preconditioner timing (100 views
    # over 360 degrees, 1024 bins over a detector 3x the image width: bins
    # 1.5 pixels apart; source and detector 1024 and 512 pixels from the
    # centre), TV, ell = 20; lambda = 2e-3, the smallest of {2e-4, 2e-3,
    # 1e-2, 5e-2} at which plain APG reaches the 1e-4 gap within 6000 its.
    "fan512_tv_f32": Workload(
        "fan512_tv_f32", "fan", 512, "tv", 2e-3, 20, "f32", "f32",
        views=100, bins=1024, noise_rel_max=0.01, outer=200, inner=20,
        fan=(1024.0, 512.0, 1.5)),
    # 256^2 CT for the unrolled solver, 180 views x 367 bins, TV, ell = 48.
    "ct256_tv_unrolled": Workload(
        "ct256_tv_unrolled", "ct", 256, "tv", 2e-4, 48, "f32", "f32",
        views=180, bins=367, noise_rel_max=0.01, outer=20, inner=20),
    # l_1 - l_1 deblurring by IRM (Alg. 2) with CG or Nystrom-PCG per outer
    # iteration: 9x9 Gaussian PSF sigma 1.6, 5 % salt + 5 % pepper, p = q = 1,
    # sketch size 100, PCG tolerance 1e-4, 20 IRM iterations; lambda and eps
    # from a PSNR grid search (lambda in {1e-3, 2e-3, 5e-3, 1e-2, 2e-2}, eps
    # in {1e-6, 1e-4}; best 36.8 dB at lambda = 2e-2, eps = 1e-4).
    "irm256_l1l1_f32": Workload(
        "irm256_l1l1_f32", "blur", 256, "tv_aniso", 0.02, 100, "f32", "f32",
        psf_k=9, psf_sigma=1.6, noise_sigma=0.0, salt_pepper=0.05, outer=20, inner=0,
        smooth_eps=1e-4),
    # 64 independent deblurring problems of uneven sizes solved together;
    # per-instance parameters from batch_instances (n and ell are maxima).
    "batch64_deblur_f32": Workload(
        "batch64_deblur_f32", "blur", 1024, "tv", 0.0, 64, "f32", "f32",
        noise_sigma=0.01, outer=100, inner=20, count=64),
}

BATCH_SIZES = (128, 256, 384, 512, 768, 1024)


@dataclasses.dataclass(frozen=True)
class BatchInstance:
    """One problem of the batched workload."""
    n: int
    psf_k: int
    psf_sigma: float
    lam: float
    ell: int
    seed: int


def batch_instances(count: int = 64, seed: int = 0,
                    sizes=BATCH_SIZES) -> list:
    """Draw the batched deblurring problems, each parameter independently:
    side uniform over `sizes`; PSF standard deviation U[0.8, 3]; PSF size
    uniform over the odd sizes 5, 7, ..., 15; TV weight U[5e-4, 5e-3];
    sketch size uniform over {16, 32, 64}.
    """
    g = rng(seed, 6)
    out = []
    for i in range(count):
        n = int(g.choice(np.asarray(sizes)))
        sigma = float(g.uniform(0.8, 3.0))
        k = int(g.choice(np.asarray((5, 7, 9, 11, 13, 15))))
        lam = float(g.uniform(5e-4, 5e-3))
        ell = int(g.choice(np.asarray((16, 32, 64))))
        out.append(BatchInstance(n, k, sigma, lam, ell, 1000 * seed + i))
    return out


def workload(name: str, **overrides) -> Workload:
    """Look up a workload and optionally shrink it (tests use small sizes)."""
    return dataclasses.replace(WORKLOADS[name], **overrides)

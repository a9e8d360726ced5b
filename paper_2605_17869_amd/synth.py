"""Seeded synthetic inputs for the SIFT extraction path.

This module only makes inputs: grayscale float32 images in [0, 1] built from
random isotropic Gaussian blobs plus low-passed Gaussian noise, affine-warped
copies for matching pairs, and Poisson arrival schedules for the serving form.
It holds none of the extraction arithmetic; both the HIP path and the FP64
oracle consume what it produces.

Recipe (all randomness from ``numpy.random.default_rng(seed)``, PCG64):

* blob centres ``cx ~ U[0, W)``, ``cy ~ U[0, H)``, widths ``s ~ U[1.5, 12]`` px,
  amplitudes ``a ~ U[-0.5, 0.5]``, drawn in that order, one vector each;
* ``img = 0.5 + sum_b a_b * exp(-((x-cx_b)^2 + (y-cy_b)^2) / (2 s_b^2))`` in
  float64, each blob evaluated inside a box of +-ceil(5 s_b) px around
  ``(floor(cx_b), floor(cy_b))``;
* noise ``N(0, 0.02)`` per pixel (std taken before filtering), low-passed by a
  separable Gaussian of sigma 0.7 truncated at radius 3 with mirrored
  (reflect-101) borders;
* ``clip(img + noise, 0, 1)`` rounded to float32.

The seed of image ``k`` of workload ``n`` is ``1_000_000 * n + k``; warped
copies add ``500_000``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NOISE_STD = 0.02
NOISE_SIGMA = 0.7
NOISE_RADIUS = 3


def workload_seed(workload_no: int, index: int, warped: bool = False) -> int:
    return 1_000_000 * int(workload_no) + int(index) + (500_000 if warped else 0)


def _mirror_index(i: np.ndarray, n: int) -> np.ndarray:
    if n == 1:
        return np.zeros_like(i)
    period = 2 * (n - 1)
    m = np.abs(i) % period
    return np.where(m >= n, period - m, m)


def _noise_lowpass(noise: np.ndarray) -> np.ndarray:
    t = np.arange(-NOISE_RADIUS, NOISE_RADIUS + 1, dtype=np.float64)
    g = np.exp(-(t * t) / (2.0 * NOISE_SIGMA * NOISE_SIGMA))
    g /= g.sum()
    h, w = noise.shape
    out = np.zeros_like(noise)
    cols = np.arange(w)
    for k, tap in enumerate(g):
        out += tap * noise[:, _mirror_index(cols + k - NOISE_RADIUS, w)]
    res = np.zeros_like(out)
    rows = np.arange(h)
    for k, tap in enumerate(g):
        res += tap * out[_mirror_index(rows + k - NOISE_RADIUS, h), :]
    return res


def blob_image(seed: int, height: int, width: int, n_blobs: int) -> np.ndarray:
    """One blob+noise image, float32, shape (height, width), values in [0, 1]."""
    if height < 1 or width < 1:
        raise ValueError("image dimensions must be positive")
    rng = np.random.default_rng(seed)
    cx = rng.uniform(0.0, width, n_blobs)
    cy = rng.uniform(0.0, height, n_blobs)
    s = rng.uniform(1.5, 12.0, n_blobs)
    a = rng.uniform(-0.5, 0.5, n_blobs)
    img = np.full((height, width), 0.5, dtype=np.float64)
    for b in range(n_blobs):
        half = int(math.ceil(5.0 * s[b]))
        x_lo = max(0, int(math.floor(cx[b])) - half)
        x_hi = min(width, int(math.floor(cx[b])) + half + 1)
        y_lo = max(0, int(math.floor(cy[b])) - half)
        y_hi = min(height, int(math.floor(cy[b])) + half + 1)
        if x_lo >= x_hi or y_lo >= y_hi:
            continue
        xs = np.arange(x_lo, x_hi, dtype=np.float64) - cx[b]
        ys = np.arange(y_lo, y_hi, dtype=np.float64) - cy[b]
        inv = 1.0 / (2.0 * s[b] * s[b])
        img[y_lo:y_hi, x_lo:x_hi] += a[b] * np.outer(np.exp(-ys * ys * inv),
                                                     np.exp(-xs * xs * inv))
    noise = rng.normal(0.0, NOISE_STD, (height, width))
    img += _noise_lowpass(noise)
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def warped_copy(img: np.ndarray, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Affine copy of ``img`` about its centre: rotation U[0,360) deg, scale
    U[0.5, 2], inverse-mapped bilinear, fill 0.5, same canvas.

    Returns the warped float32 image and the 2x3 forward map A (dst = A @ [x, y, 1]).
    """
    rng = np.random.default_rng(seed)
    ang = math.radians(rng.uniform(0.0, 360.0))
    scale = rng.uniform(0.5, 2.0)
    h, w = img.shape
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    c, s = math.cos(ang) * scale, math.sin(ang) * scale
    fwd = np.array([[c, -s, cx - c * cx + s * cy],
                    [s, c, cy - s * cx - c * cy]], dtype=np.float64)
    # inverse map: src = M^-1 (dst - t)
    m = fwd[:, :2]
    inv = np.linalg.inv(m)
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    dx = xx - fwd[0, 2]
    dy = yy - fwd[1, 2]
    sx = inv[0, 0] * dx + inv[0, 1] * dy
    sy = inv[1, 0] * dx + inv[1, 1] * dy
    x0 = np.floor(sx)
    y0 = np.floor(sy)
    fx = sx - x0
    fy = sy - y0
    x0 = x0.astype(np.int64)
    y0 = y0.astype(np.int64)
    src = img.astype(np.float64)

    def tap(yi, xi):
        ok = (yi >= 0) & (yi < h) & (xi >= 0) & (xi < w)
        v = np.full(yi.shape, 0.5)
        v[ok] = src[yi[ok], xi[ok]]
        return v

    out = ((1 - fy) * ((1 - fx) * tap(y0, x0) + fx * tap(y0, x0 + 1))
           + fy * ((1 - fx) * tap(y0 + 1, x0) + fx * tap(y0 + 1, x0 + 1)))
    return np.clip(out, 0.0, 1.0).astype(np.float32), fwd


def poisson_arrivals(seed: int, n: int, qps: float) -> np.ndarray:
    """Arrival times (s) of ``n`` requests with exponential inter-arrival gaps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, n))


# ---------------------------------------------------------------------------
# Workload recipes: image sizes, blob counts and SIFT settings of each
# benchmark workload.  Settings are plain numbers; each side builds its own
# parameter object from them.

BASE_SETTINGS = dict(
    n_octaves=4, n_scales=3, upsample=0, sigma0=1.6, sigma_in=0.5,
    contrast_threshold=0.04 / 3.0, prefilter_ratio=0.5, edge_ratio=10.0,
    border=5, refine_iters=5, ori_bins=36, ori_sigma_factor=1.5,
    ori_radius_factor=3.0, ori_peak_ratio=0.8, upright=0, desc_width=4,
    desc_ori_bins=8, desc_magnif=3.0, desc_clamp=0.2, dsp_scales=(1.0,),
    rootsift=0, max_keypoints=65536,
)

# Blob density of the 1024x768 / 1000-blob workload, reused where a workload
# only says "same generator".
BLOB_DENSITY = 1000.0 / (1024 * 768)


def dsp_linspace(k: int = 10, lo: float = 1.0 / 6.0, hi: float = 4.0 / 3.0) -> tuple:
    return tuple(float(v) for v in np.linspace(lo, hi, k))


@dataclass
class Workload:
    number: int
    name: str
    sizes: list            # list of (height, width)
    n_blobs: list          # per image
    settings: dict = field(default_factory=dict)
    warped_pairs: bool = False

    def image(self, k: int) -> np.ndarray:
        h, w = self.sizes[k]
        return blob_image(workload_seed(self.number, k), h, w, self.n_blobs[k])

    def images(self) -> list:
        out = [self.image(k) for k in range(len(self.sizes))]
        if self.warped_pairs:
            out += [warped_copy(out[k], workload_seed(self.number, k, True))[0]
                    for k in range(len(self.sizes))]
        return out


def workload(number: int, n_images: int | None = None) -> Workload:
    """Workload ``number`` in 1..5 (optionally with fewer images)."""
    s = dict(BASE_SETTINGS)
    if number == 1:
        wl = Workload(1, "single 640x480, 200 blobs, per-image path",
                      [(480, 640)], [200], s)
    elif number == 2:
        s.update(upsample=1)
        n = 64 if n_images is None else n_images
        wl = Workload(2, f"batch of {n} x 1024x768, 1000 blobs, upsampled octave -1",
                      [(768, 1024)] * n, [1000] * n, s)
    elif number == 3:
        s.update(max_keypoints=8192)
        n = 16 if n_images is None else max(1, n_images // 2)
        sizes = [(1066, 1600)] * n + [(1600, 1066)] * n
        wl = Workload(3, f"{2 * n} x 1600x1066 / 1066x1600, 4000 blobs, + warped copies",
                      sizes, [4000] * (2 * n), s, warped_pairs=True)
    elif number == 4:
        s.update(max_keypoints=8192)
        n = 2200 if n_images is None else n_images
        rng = np.random.default_rng(workload_seed(4, 999_999))
        ws = rng.integers(320, 2049, max(n, 2200))[:n]
        hs = rng.integers(320, 2049, max(n, 2200))[:n]
        sizes = [(int(h), int(w)) for h, w in zip(hs, ws)]
        blobs = [max(1, int(round(h * w * BLOB_DENSITY))) for h, w in sizes]
        wl = Workload(4, "serving: Poisson arrivals, W,H ~ U[320,2048]", sizes, blobs, s)
    elif number == 5:
        s.update(dsp_scales=dsp_linspace(), rootsift=1)
        n = 256 if n_images is None else n_images
        rng = np.random.default_rng(workload_seed(5, 999_999))
        ws = rng.integers(600, 1201, max(n, 256))[:n]
        hs = rng.integers(400, 901, max(n, 256))[:n]
        sizes = [(int(h), int(w)) for h, w in zip(hs, ws)]
        blobs = [max(1, int(round(h * w * BLOB_DENSITY))) for h, w in sizes]
        wl = Workload(5, "DSP-SIFT: 256 images U[600,1200]xU[400,900], K=10, RootSIFT",
                      sizes, blobs, s)
    else:
        raise ValueError(f"no workload {number}")
    return wl


def descriptor_sets(seed: int, n_a: int, n_b: int, n_common: int, noise: float = 0.05,
                    dim: int = 128) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Seeded descriptor sets shaped like SIFT output: non-negative unit rows.

    Rows of ``a`` are |N(0, 1)| vectors normalised to unit length.  ``b`` holds
    ``n_common`` of them (a random subset, in random order), each perturbed by
    |N(0, noise)| and renormalised, and ``n_b - n_common`` fresh rows.  Returns
    (a, b, truth) with truth[k] = (row of a, row of b) for the common rows.
    float32 throughout; no part of matching is computed here."""
    rng = np.random.default_rng(seed)

    def unit(x):
        x = np.abs(x)
        return x / np.linalg.norm(x, axis=1, keepdims=True)

    if not 0 <= n_common <= min(n_a, n_b):
        raise ValueError("n_common must be in 0..min(n_a, n_b)")
    a = unit(rng.normal(size=(n_a, dim)))
    src = rng.permutation(n_a)[:n_common]
    dst = rng.permutation(n_b)[:n_common]
    b = unit(rng.normal(size=(n_b, dim)))
    b[dst] = unit(a[src] + np.abs(rng.normal(0.0, noise, size=(n_common, dim))))
    truth = np.stack([src, dst], axis=1) if n_common else np.zeros((0, 2), dtype=np.int64)
    return a.astype(np.float32), b.astype(np.float32), truth.astype(np.int64)


def homography_pairs(seed: int, n: int, outlier_frac: float = 0.3, noise: float = 0.5,
                     size: tuple = (1066, 1600)) -> tuple:
    """Seeded correspondences under a random homography: points uniform in an
    H x W image, a random homography near a similarity (rotation U[0, 360),
    scale U[0.5, 2], a small perspective term) about the image centre, inlier
    targets perturbed by N(0, noise) px, outlier targets uniform in the image.
    Returns (a, b, H, inlier_mask) as float64 / bool."""
    rng = np.random.default_rng(seed)
    h, w = size
    a = np.stack([rng.uniform(0, w, n), rng.uniform(0, h, n)], axis=1)
    ang = rng.uniform(0.0, 2.0 * math.pi)
    sc = rng.uniform(0.5, 2.0)
    cx, cy = (w - 1) / 2.0, (h - 1) / 2.0
    c, s = math.cos(ang) * sc, math.sin(ang) * sc
    H = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    H[2, :2] = rng.uniform(-2e-4, 2e-4, 2)
    T1 = np.array([[1.0, 0.0, -cx], [0.0, 1.0, -cy], [0.0, 0.0, 1.0]])
    T2 = np.array([[1.0, 0.0, cx], [0.0, 1.0, cy], [0.0, 0.0, 1.0]])
    H = T2 @ H @ T1
    H /= H[2, 2]
    ah = np.c_[a, np.ones(n)] @ H.T
    b = ah[:, :2] / ah[:, 2:3] + rng.normal(0.0, noise, (n, 2))
    out = rng.uniform(size=n) < outlier_frac
    b[out] = np.stack([rng.uniform(0, w, out.sum()), rng.uniform(0, h, out.sum())], axis=1)
    return a, b, H, ~out


def sample_numbers(seed: int, k: int = 1500) -> np.ndarray:
    """The random numbers a verification draws its k minimal samples from:
    k x 4 float32 values in [0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.random((k, 4), dtype=np.float32)

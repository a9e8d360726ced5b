"""FP64 CPU oracle of the SIFT extraction path.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
reference that the HIP path is checked against.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does.  It shares no code with the HIP library.

Everything is computed in float64 from the float32 input image.  The steps
follow the pipeline the paper names in its method section (Eq. (1): pyramid ->
DoG -> extrema -> orientation -> descriptor; section 3.2 "GPU Pipeline
Stages" and "DSP Multi-Scale Descriptor Pooling" / "RootSIFT Normalization")
and, where the paper defers to it, Lowe's SIFT (IJCV 2004).  Where the paper is
silent the reading taken is stated at the function that applies it.

Every accept/reject decision on the way is logged with a relative margin so a
checker can tell a decisive outcome from one that a rounding change could flip.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, fields, replace

import numpy as np

TWO_PI = 2.0 * math.pi


# ---------------------------------------------------------------------------
# Parameters

@dataclass
class Params:
    """SIFT settings.  Defaults: 4 octaves, 3 scales per octave, sigma0 1.6,
    no upsampled octave, contrast threshold 0.04/3, edge ratio 10, 36-bin
    orientation histogram, 4x4x8 descriptor with 0.2 clamp."""
    n_octaves: int = 4            # octaves 0..n_octaves-1 (octave -1 extra if upsample)
    n_scales: int = 3             # s: DoG layers searched per octave
    upsample: int = 0             # 1: add octave -1 from a 2x bilinear upsample
    sigma0: float = 1.6
    sigma_in: float = 0.5         # blur assumed present in the input image
    contrast_threshold: float = 0.04 / 3.0
    prefilter_ratio: float = 0.5  # candidate pre-gate |D| > ratio * threshold
    edge_ratio: float = 10.0
    border: int = 5
    refine_iters: int = 5
    ori_bins: int = 36
    ori_sigma_factor: float = 1.5
    ori_radius_factor: float = 3.0
    ori_peak_ratio: float = 0.8
    upright: int = 0
    desc_width: int = 4
    desc_ori_bins: int = 8
    desc_magnif: float = 3.0
    desc_clamp: float = 0.2
    dsp_scales: tuple = (1.0,)
    rootsift: int = 0
    max_keypoints: int = 65536
    max_candidates: int = 65536   # detections refined, first ones in canonical order
    upsample_max_pixels: int = 0  # > 0: no octave -1 for images of more pixels than this
    pyramid_fp16: int = 0         # 1: levels of every octave after the first stored as fp16

    @classmethod
    def from_settings(cls, settings: dict) -> "Params":
        names = {f.name for f in fields(cls)}
        kw = {k: v for k, v in settings.items() if k in names}
        if "dsp_scales" in kw:
            kw["dsp_scales"] = tuple(float(v) for v in kw["dsp_scales"])
        return cls(**kw)


# ---------------------------------------------------------------------------
# Small helpers

def round_half_away(x: float) -> int:
    """Round to nearest, ties away from zero (never Python's ties-to-even)."""
    return int(math.copysign(math.floor(abs(x) + 0.5), x))


def mirror_index(i, n: int):
    """Reflect-101 border (... c b | a b c ... : index -1 -> 1), repeated with
    period 2(n-1) for indices far outside; n == 1 maps everything to 0."""
    i = np.asarray(i)
    if n == 1:
        return np.zeros_like(i)
    period = 2 * (n - 1)
    m = np.abs(i) % period
    return np.where(m >= n, period - m, m)


# ---------------------------------------------------------------------------
# Scale space (section 3.2: separable Gaussian convolution with 4-sigma
# truncation; DoG by subtraction of adjacent levels)

def gaussian_taps(sigma: float):
    """Normalised sampled Gaussian g[t] ~ exp(-t^2 / (2 sigma^2)), t = -R..R,
    R = ceil(4 sigma) (the paper's 4-sigma truncation, read as a ceiling)."""
    radius = int(math.ceil(4.0 * sigma))
    t = np.arange(-radius, radius + 1, dtype=np.float64)
    g = np.exp(-(t * t) / (2.0 * sigma * sigma))
    return radius, g / g.sum()


def correlate_rows(img: np.ndarray, g: np.ndarray) -> np.ndarray:
    """out[r, c] = sum_t g[t] * img[r, mirror(c + t - R)] (horizontal pass)."""
    radius = (len(g) - 1) // 2
    w = img.shape[1]
    cols = np.arange(w)
    out = np.zeros_like(img, dtype=np.float64)
    for k in range(len(g)):
        out += g[k] * img[:, mirror_index(cols + k - radius, w)]
    return out


def correlate_cols(img: np.ndarray, g: np.ndarray) -> np.ndarray:
    """out[r, c] = sum_t g[t] * img[mirror(r + t - R), c] (vertical pass)."""
    radius = (len(g) - 1) // 2
    h = img.shape[0]
    rows = np.arange(h)
    out = np.zeros_like(img, dtype=np.float64)
    for k in range(len(g)):
        out += g[k] * img[mirror_index(rows + k - radius, h), :]
    return out


def gaussian_blur(img: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian: horizontal pass, then vertical pass."""
    _, g = gaussian_taps(sigma)
    return correlate_cols(correlate_rows(np.asarray(img, dtype=np.float64), g), g)


def upsample2x(img: np.ndarray) -> np.ndarray:
    """Octave -1 base (the paper's 2x input magnification): bilinear samples
    U[i, j] = I(y = i/2, x = j/2), size 2H x 2W, the row/column past the last
    one clamped to it."""
    src = np.asarray(img, dtype=np.float64)
    h, w = src.shape
    ys = np.arange(2 * h) / 2.0
    xs = np.arange(2 * w) / 2.0
    y0 = np.floor(ys).astype(np.int64)
    x0 = np.floor(xs).astype(np.int64)
    fy = (ys - y0)[:, None]
    fx = (xs - x0)[None, :]
    y1 = np.minimum(y0 + 1, h - 1)
    x1 = np.minimum(x0 + 1, w - 1)
    a = src[y0][:, x0]
    b = src[y0][:, x1]
    c = src[y1][:, x0]
    d = src[y1][:, x1]
    return (1 - fy) * ((1 - fx) * a + fx * b) + fy * ((1 - fx) * c + fx * d)


def level_sigmas(p: Params):
    """(sigma of the initial blur, [incremental sigma of levels 1..s+2]).

    Level i of an octave carries total blur sigma0 * k^i, k = 2^(1/s); level i
    is made from level i-1 by a blur of sigma0 * sqrt(k^(2i) - k^(2(i-1))).
    The base of the first octave already carries sigma_in (2 sigma_in after
    upsampling), so its initial blur is sqrt(sigma0^2 - assumed^2)."""
    s = p.n_scales
    assumed = p.sigma_in * (2.0 if p.upsample else 1.0)
    sigma_init = math.sqrt(max(p.sigma0 ** 2 - assumed ** 2, 0.01))
    k2 = 2.0 ** (2.0 / s)
    incs = []
    for i in range(1, s + 3):
        incs.append(p.sigma0 * math.sqrt(k2 ** i - k2 ** (i - 1)))
    return sigma_init, incs


@dataclass
class Octave:
    o: int                 # octave index (-1 for the upsampled octave)
    L: np.ndarray          # (s+3, h, w) Gaussian levels
    D: np.ndarray          # (s+2, h, w) DoG layers, D[i] = L[i+1] - L[i]

    @property
    def shape(self):
        return self.L.shape[1:]


def octave_shapes(height: int, width: int, p: Params):
    h, w = (2 * height, 2 * width) if p.upsample else (height, width)
    shapes = []
    for _ in range(p.n_octaves + (1 if p.upsample else 0)):
        shapes.append((h, w))
        h, w = (h + 1) // 2, (w + 1) // 2
    return shapes


def effective_params(height: int, width: int, p: Params) -> Params:
    """The settings an image is extracted with.  The paper's VRAM-adaptive
    execution drops the 2x upsampled base for inputs above a size (4 MP on
    its 4 GB GPU): with upsample_max_pixels > 0, an image of more pixels than
    that is processed exactly as with upsample = 0."""
    if p.upsample and p.upsample_max_pixels > 0 and height * width > p.upsample_max_pixels:
        return replace(p, upsample=0)
    return p


def check_size(height: int, width: int, p: Params):
    last = octave_shapes(height, width, p)[-1]
    if min(last) < 2 * p.border + 3:
        raise ValueError(f"image {height}x{width} too small for {p.n_octaves} octaves")


def store_fp16(level: np.ndarray) -> np.ndarray:
    """A level as held in fp16 storage (section 3.2, "GPU Pipeline Stages":
    fp16 storage with fp32 compute, the first octave kept in fp32): the value
    relative to mid-grey, L - 1/2, rounded to the nearest fp16 (ties to even),
    read back as L.  Holding levels relative to mid-grey is this
    implementation's storage convention; it changes no difference of levels."""
    return (level - 0.5).astype(np.float16).astype(np.float64) + 0.5


def scale_space(img: np.ndarray, p: Params) -> list:
    """Gaussian and DoG pyramid.  The next octave's level 0 is level s of the
    current octave taken at every second pixel, with no further blur.  With
    pyramid_fp16, every level of the octaves after the first is stored in fp16
    (store_fp16) as soon as it is made, and the next level is blurred from the
    stored value."""
    img = np.asarray(img, dtype=np.float32).astype(np.float64)
    p = effective_params(img.shape[0], img.shape[1], p)
    check_size(img.shape[0], img.shape[1], p)
    sigma_init, incs = level_sigmas(p)
    base = upsample2x(img) if p.upsample else img
    level0 = gaussian_blur(base, sigma_init)
    o0 = -1 if p.upsample else 0
    octaves = []
    for o in range(o0, o0 + p.n_octaves + (1 if p.upsample else 0)):
        store = store_fp16 if (p.pyramid_fp16 and o > o0) else (lambda x: x)
        levels = [store(level0)]
        for sig in incs:
            levels.append(store(gaussian_blur(levels[-1], sig)))
        L = np.stack(levels)
        D = L[1:] - L[:-1]
        octaves.append(Octave(o, L, D))
        level0 = L[p.n_scales][0::2, 0::2]
    return octaves


# ---------------------------------------------------------------------------
# Extrema (section 3.2: 26-neighbour comparison with contrast gating)

NEIGHBOURS = [(di, dr, dc) for di in (-1, 0, 1) for dr in (-1, 0, 1)
              for dc in (-1, 0, 1) if (di, dr, dc) != (0, 0, 0)]


def candidate_mask(D: np.ndarray, i: int, p: Params) -> np.ndarray:
    """Boolean (h, w) mask of layer i: |D| > prefilter_ratio * threshold and
    D strictly above all 26 neighbours or strictly below all of them, for
    border <= r < h - border, border <= c < w - border."""
    _, h, w = D.shape
    b = p.border
    thr = p.prefilter_ratio * p.contrast_threshold
    ctr = D[i, b:h - b, b:w - b]
    is_max = np.ones_like(ctr, dtype=bool)
    is_min = np.ones_like(ctr, dtype=bool)
    for di, dr, dc in NEIGHBOURS:
        nb = D[i + di, b + dr:h - b + dr, b + dc:w - b + dc]
        is_max &= ctr > nb
        is_min &= ctr < nb
    mask = np.zeros((h, w), dtype=bool)
    mask[b:h - b, b:w - b] = (np.abs(ctr) > thr) & (is_max | is_min)
    return mask


def pixel_margins(D: np.ndarray, i: int, r: int, c: int, p: Params) -> dict:
    """Relative margins of the candidate decision at one pixel: m_pre for the
    pre-gate, m_ext for the 26-neighbour test (for a pixel that is not an
    extremum: how far the nearest neighbour is from making it one)."""
    thr = p.prefilter_ratio * p.contrast_threshold
    v = D[i, r, c]
    diffs = np.array([v - D[i + di, r + dr, c + dc] for di, dr, dc in NEIGHBOURS])
    scale = max(abs(v), 1e-300)
    if np.all(diffs > 0) or np.all(diffs < 0):
        m_ext = float(np.min(np.abs(diffs)) / scale)
    else:
        # to become a max every non-positive diff must turn positive; likewise min
        to_max = float(np.max(np.maximum(-diffs, 0.0)))
        to_min = float(np.max(np.maximum(diffs, 0.0)))
        m_ext = min(to_max, to_min) / scale
    return dict(m_pre=abs(abs(v) - thr) / thr, m_ext=m_ext)


def detect(octaves: list, p: Params) -> list:
    """Candidates in canonical order (octave, layer, row, column), ascending."""
    out = []
    for oc in octaves:
        for i in range(1, p.n_scales + 1):
            rows, cols = np.nonzero(candidate_mask(oc.D, i, p))
            for r, c in zip(rows.tolist(), cols.tolist()):
                out.append((oc.o, i, r, c))
    return out


# ---------------------------------------------------------------------------
# Sub-pixel refinement (section 3.2: 3-D Taylor expansion solved by Cramer's
# rule, up to 5 iterations, Hessian edge rejection)

def derivatives(D: np.ndarray, i: int, r: int, c: int):
    """Central-difference gradient (dx, dy, ds) and Hessian of D at (i, r, c);
    x runs along columns, y along rows, s along layers."""
    v = D[i, r, c]
    dx = (D[i, r, c + 1] - D[i, r, c - 1]) * 0.5
    dy = (D[i, r + 1, c] - D[i, r - 1, c]) * 0.5
    ds = (D[i + 1, r, c] - D[i - 1, r, c]) * 0.5
    dxx = D[i, r, c + 1] + D[i, r, c - 1] - 2.0 * v
    dyy = D[i, r + 1, c] + D[i, r - 1, c] - 2.0 * v
    dss = D[i + 1, r, c] + D[i - 1, r, c] - 2.0 * v
    dxy = (D[i, r + 1, c + 1] - D[i, r + 1, c - 1]
           - D[i, r - 1, c + 1] + D[i, r - 1, c - 1]) * 0.25
    dxs = (D[i + 1, r, c + 1] - D[i + 1, r, c - 1]
           - D[i - 1, r, c + 1] + D[i - 1, r, c - 1]) * 0.25
    dys = (D[i + 1, r + 1, c] - D[i + 1, r - 1, c]
           - D[i - 1, r + 1, c] + D[i - 1, r - 1, c]) * 0.25
    g = np.array([dx, dy, ds])
    H = np.array([[dxx, dxy, dxs], [dxy, dyy, dys], [dxs, dys, dss]])
    return float(v), g, H


def det3(m: np.ndarray) -> float:
    return float(m[0, 0] * (m[1, 1] * m[2, 2] - m[1, 2] * m[2, 1])
                 - m[0, 1] * (m[1, 0] * m[2, 2] - m[1, 2] * m[2, 0])
                 + m[0, 2] * (m[1, 0] * m[2, 1] - m[1, 1] * m[2, 0]))


def cramer_solve(H: np.ndarray, b: np.ndarray):
    """Solve H x = b by Cramer's rule: x_k = det(H with column k := b) / det H.
    Returns (x, det H); x is None when det H == 0."""
    det = det3(H)
    if det == 0.0:
        return None, det
    x = np.empty(3)
    for k in range(3):
        mk = H.copy()
        mk[:, k] = b
        x[k] = det3(mk) / det
    return x, det


def _half_margin(d: float) -> float:
    """Relative distance of |x| to the nearest rounding boundary k + 1/2."""
    h = math.floor(d) + 0.5
    return abs(d - h) / h


def refine(oc: Octave, i: int, r: int, c: int, p: Params) -> dict:
    """Newton steps on D from candidate (i, r, c) of octave oc.

    Reading of the step rule: a step is accepted when every |x^| <= 0.5; else
    each coordinate with |x^| > 0.5 moves by x^ rounded half away from zero,
    and the candidate is dropped when it leaves layers [1, s] or the border
    frame, when H is singular, or when refine_iters solves did not converge.
    Then |D(x^)| >= threshold (contrast) and the 2x2 spatial Hessian must have
    det > 0 and tr^2 * r < (r + 1)^2 * det (edge test)."""
    D = oc.D
    _, h, w = D.shape
    s, b = p.n_scales, p.border
    res = dict(o=oc.o, i0=i, r0=r, c0=c, status="", m_move=math.inf)
    converged = False
    for _ in range(p.refine_iters):
        v, g, H = derivatives(D, i, r, c)
        x, det = cramer_solve(H, -g)
        if x is None or not np.all(np.isfinite(x)):
            res["status"] = "singular"
            return res
        for k in range(3):
            res["m_move"] = min(res["m_move"], _half_margin(abs(x[k])))
        if np.max(np.abs(x)) <= 0.5:
            converged = True
            break
        moves = [round_half_away(x[k]) if abs(x[k]) > 0.5 else 0 for k in range(3)]
        c += moves[0]
        r += moves[1]
        i += moves[2]
        if i < 1 or i > s or r < b or r >= h - b or c < b or c >= w - b:
            res["status"] = "bounds"
            return res
    if not converged:
        res["status"] = "no_converge"
        return res
    contrast = v + 0.5 * float(np.dot(g, x))
    thr = p.contrast_threshold
    res["m_con"] = abs(abs(contrast) - thr) / thr
    res.update(i=i, r=r, c=c, xhat=x.copy(), contrast=contrast)
    if abs(contrast) < thr:
        res["status"] = "contrast"
        return res
    dxx, dyy, dxy = H[0, 0], H[1, 1], H[0, 1]
    tr = dxx + dyy
    det2 = dxx * dyy - dxy * dxy
    re = p.edge_ratio
    if det2 <= 0.0:
        res["m_edge"] = abs(det2) / max(abs(dxx * dyy) + dxy * dxy, 1e-300)
        res["status"] = "edge"
        return res
    lhs, rhs = tr * tr * re, (re + 1.0) ** 2 * det2
    res["m_edge"] = min(abs(rhs - lhs) / rhs, det2 / (abs(dxx * dyy) + dxy * dxy))
    if lhs >= rhs:
        res["status"] = "edge"
        return res
    scale = 2.0 ** oc.o
    sigma_oct = p.sigma0 * 2.0 ** ((i + x[2]) / s)
    res.update(status="ok", x_oct=c + x[0], y_oct=r + x[1], sigma_oct=sigma_oct,
               x=(c + x[0]) * scale, y=(r + x[1]) * scale, sigma=sigma_oct * scale,
               response=abs(contrast))
    return res


# ---------------------------------------------------------------------------
# Gradients shared by the orientation and descriptor stages

def gradients(L: np.ndarray, rr: np.ndarray, cc: np.ndarray):
    """Magnitude and angle in [0, 2 pi) of the central-difference gradient
    (gx = L[r, c+1] - L[r, c-1], gy = L[r+1, c] - L[r-1, c]; y points down)."""
    gx = L[rr, cc + 1] - L[rr, cc - 1]
    gy = L[rr + 1, cc] - L[rr - 1, cc]
    mag = np.sqrt(gx * gx + gy * gy)
    ang = np.arctan2(gy, gx)
    ang = np.where(ang < 0.0, ang + TWO_PI, ang)
    return mag, ang


def _window(L: np.ndarray, r: int, c: int, radius: int):
    """Integer pixels of the square [-radius, radius]^2 around (r, c) whose
    central differences stay inside the level (rows 1..h-2, cols 1..w-2)."""
    h, w = L.shape
    dr, dc = np.meshgrid(np.arange(-radius, radius + 1), np.arange(-radius, radius + 1),
                         indexing="ij")
    dr, dc = dr.ravel(), dc.ravel()
    rr, cc = r + dr, c + dc
    ok = (rr >= 1) & (rr <= h - 2) & (cc >= 1) & (cc <= w - 2)
    return dr[ok], dc[ok], rr[ok], cc[ok]


# ---------------------------------------------------------------------------
# Orientation (section 3.2: 36-bin histogram, [1/4, 1/2, 1/4] smoothing,
# parabolic sub-bin refinement)

def orientation_histogram(L: np.ndarray, r: int, c: int, sigma_oct: float, p: Params):
    """Raw histogram of magnitude x Gaussian(ori_sigma_factor * sigma) weights
    over the square window of radius floor(ori_radius_factor * sigma_w + 1/2)
    centred on the integer pixel (r, c).  Reading: each sample is split
    linearly between the two nearest bins (bin j centred at angle j*360/n)."""
    n = p.ori_bins
    sw = p.ori_sigma_factor * sigma_oct
    q = p.ori_radius_factor * sw + 0.5
    radius = int(math.floor(q))
    m_rad = abs(q - round(q)) / q
    dr, dc, rr, cc = _window(L, r, c, radius)
    mag, ang = gradients(L, rr, cc)
    wgt = np.exp(-(dr * dr + dc * dc) / (2.0 * sw * sw)) * mag
    pos = ang * (n / TWO_PI)
    j0 = np.floor(pos)
    f = pos - j0
    j0 = j0.astype(np.int64)
    hist = np.zeros(n)
    np.add.at(hist, j0 % n, wgt * (1.0 - f))
    np.add.at(hist, (j0 + 1) % n, wgt * f)
    return hist, m_rad


def orientation_peaks(hist: np.ndarray, p: Params):
    """One circular [1/4, 1/2, 1/4] smoothing pass, then every bin that is
    strictly above both neighbours and >= ori_peak_ratio * max, ascending, each
    refined by the vertex of the parabola through it and its neighbours.
    Returns (angles in degrees, margin of the peak decisions)."""
    n = len(hist)
    hs = 0.25 * np.roll(hist, 1) + 0.5 * hist + 0.25 * np.roll(hist, -1)
    hmax = float(hs.max())
    if hmax <= 0.0:
        return [], 0.0
    left, right = np.roll(hs, 1), np.roll(hs, -1)
    angles = []
    m_peak = math.inf
    for j in range(n):
        lp = min(hs[j] - left[j], hs[j] - right[j]) / hmax
        rm = (hs[j] - p.ori_peak_ratio * hmax) / hmax
        if lp > 0.0 and rm >= 0.0:
            m_peak = min(m_peak, lp, rm)
            denom = left[j] - 2.0 * hs[j] + right[j]
            delta = 0.5 * (left[j] - right[j]) / denom
            ang = (j + delta) * (360.0 / n)
            ang = ang % 360.0
            angles.append(float(ang))
        else:
            fails = [abs(m) for m, ok in ((lp, lp > 0.0), (rm, rm >= 0.0)) if not ok]
            m_peak = min(m_peak, max(fails))
    return angles, m_peak


# ---------------------------------------------------------------------------
# Descriptor (4x4x8 gradient histogram; DSP pooling over domain sizes and
# RootSIFT from section 3.2)

def raw_descriptor(L: np.ndarray, r: int, c: int, x_oct: float, y_oct: float,
                   sigma_oct: float, angle_deg: float, scale: float, p: Params) -> np.ndarray:
    """Unnormalised d x d x n histogram at one domain size.

    Cells are desc_magnif * sigma * scale px wide on a grid rotated by the
    keypoint angle and centred on the sub-pixel position; each sample adds
    magnitude x exp(-(x_r^2 + y_r^2) / (2 (d/2)^2)) trilinearly to the two
    nearest cells along each grid axis and the two nearest orientation bins.
    Index = (row * d + col) * n + orientation."""
    d, n = p.desc_width, p.desc_ori_bins
    th = math.radians(angle_deg)
    ct, st = math.cos(th), math.sin(th)
    wc = p.desc_magnif * sigma_oct * scale
    radius = int(math.ceil(math.sqrt(2.0) * (d + 1) * 0.5 * wc))
    dr, dc, rr, cc = _window(L, r, c, radius)
    u = cc - x_oct
    v = rr - y_oct
    xr = (ct * u + st * v) / wc
    yr = (-st * u + ct * v) / wc
    cb = xr + d / 2.0 - 0.5
    rb = yr + d / 2.0 - 0.5
    ok = (rb > -1.0) & (rb < d) & (cb > -1.0) & (cb < d)
    xr, yr, cb, rb, rr, cc = xr[ok], yr[ok], cb[ok], rb[ok], rr[ok], cc[ok]
    mag, ang = gradients(L, rr, cc)
    ob = np.mod(ang - th, TWO_PI) * (n / TWO_PI)
    wgt = mag * np.exp(-(xr * xr + yr * yr) / (2.0 * (d / 2.0) ** 2))
    r0, c0, o0 = np.floor(rb), np.floor(cb), np.floor(ob)
    fr, fc, fo = rb - r0, cb - c0, ob - o0
    r0, c0, o0 = r0.astype(np.int64), c0.astype(np.int64), o0.astype(np.int64)
    hist = np.zeros(d * d * n)
    for a in (0, 1):
        wr = fr if a else 1.0 - fr
        for bb in (0, 1):
            wcol = fc if bb else 1.0 - fc
            for e in (0, 1):
                wo = fo if e else 1.0 - fo
                row, col, ori = r0 + a, c0 + bb, (o0 + e) % n
                keep = (row >= 0) & (row < d) & (col >= 0) & (col < d)
                idx = (row * d + col) * n + ori
                np.add.at(hist, idx[keep], (wgt * wr * wcol * wo)[keep])
    return hist


def normalise(hist: np.ndarray, p: Params) -> np.ndarray:
    """L2 normalise, clamp at desc_clamp, L2 normalise; then, with rootsift,
    L1 normalise and take the element-wise square root."""
    v = hist.copy()
    nrm = math.sqrt(float(np.dot(v, v)))
    v = v / nrm if nrm > 0.0 else np.zeros_like(v)
    v = np.minimum(v, p.desc_clamp)
    nrm = math.sqrt(float(np.dot(v, v)))
    v = v / nrm if nrm > 0.0 else np.zeros_like(v)
    if p.rootsift:
        l1 = float(np.sum(np.abs(v)))
        v = v / l1 if l1 > 0.0 else v
        v = np.sqrt(v)
    return v


def descriptor(L: np.ndarray, r: int, c: int, x_oct: float, y_oct: float,
               sigma_oct: float, angle_deg: float, p: Params) -> np.ndarray:
    """DSP pooling: the raw histograms of every domain size in dsp_scales are
    averaged before one normalisation (with dsp_scales = (1,) this is the plain
    descriptor)."""
    acc = np.zeros(p.desc_width * p.desc_width * p.desc_ori_bins)
    for sk in p.dsp_scales:
        acc += raw_descriptor(L, r, c, x_oct, y_oct, sigma_oct, angle_deg, sk, p)
    acc /= len(p.dsp_scales)
    return normalise(acc, p)


# ---------------------------------------------------------------------------
# Whole pipeline

KEYPOINT_DTYPE = np.dtype([
    ("x", "f8"), ("y", "f8"), ("sigma", "f8"), ("angle", "f8"), ("response", "f8"),
    ("octave", "i4"), ("layer", "i4"), ("ix", "i4"), ("iy", "i4"),
    ("src_layer", "i4"), ("src_iy", "i4"), ("src_ix", "i4"),
])


@dataclass
class Result:
    keypoints: np.ndarray          # KEYPOINT_DTYPE, canonical order, capped
    descriptors: np.ndarray        # (n, d*d*n_ori) float64
    n_found: int                   # keypoints before the cap
    log: list = field(default_factory=list)   # one dict per refined candidate
    octaves: list = field(default_factory=list)
    n_candidates: int = 0          # detections before the candidate cap


def orient_and_describe(oc: Octave, res: dict, p: Params):
    """Orientation(s) and descriptors of one refined keypoint; updates res."""
    L = oc.L[res["i"]]
    r, c = res["r"], res["c"]
    if p.upright:
        angles, res["m_peak"], res["m_rad"] = [0.0], math.inf, math.inf
    else:
        hist, res["m_rad"] = orientation_histogram(L, r, c, res["sigma_oct"], p)
        angles, res["m_peak"] = orientation_peaks(hist, p)
    res["angles"] = angles
    res["desc"] = [descriptor(L, r, c, res["x_oct"], res["y_oct"], res["sigma_oct"], a, p)
                   for a in angles]


def sift(img: np.ndarray, p: Params | None = None, keep_octaves: bool = False,
         describe: bool = True) -> Result:
    """Keypoints and descriptors of a float32 image in [0, 1].

    Keypoints come in the order of the candidate they were refined from
    (octave, layer, row, column, ascending), then by orientation bin; two
    candidates that converge to one point give two keypoints; the first
    max_keypoints are kept and n_found counts all of them.  Only the first
    max_candidates detections (same canonical order) are refined; the
    paper fixes no such capacity, so with the default none is cut on the
    workloads used here."""
    p = p or Params()
    p = effective_params(np.shape(img)[0], np.shape(img)[1], p)
    octaves = scale_space(img, p)
    by_o = {oc.o: oc for oc in octaves}
    log = []
    kps, descs = [], []
    cands = detect(octaves, p)
    for (o, i, r, c) in cands[:p.max_candidates]:
        oc = by_o[o]
        res = refine(oc, i, r, c, p)
        res.update(pixel_margins(oc.D, i, r, c, p))
        if res["status"] == "ok":
            if describe:
                orient_and_describe(oc, res, p)
            else:
                res["angles"], res["desc"] = [], []
            for k, a in enumerate(res["angles"]):
                kps.append((res["x"], res["y"], res["sigma"], a, res["response"], o,
                            res["i"], res["c"], res["r"], i, r, c))
                descs.append(res["desc"][k])
        log.append(res)
    n_found = len(kps)
    kps = kps[:p.max_keypoints]
    descs = descs[:p.max_keypoints]
    nd = p.desc_width * p.desc_width * p.desc_ori_bins
    return Result(np.array(kps, dtype=KEYPOINT_DTYPE),
                  np.array(descs, dtype=np.float64).reshape(-1, nd),
                  n_found, log, octaves if keep_octaves else [], len(cands))

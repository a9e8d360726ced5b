"""Reference geometric verification (test infrastructure only).

Plain FP64 NumPy statement of the verification step that follows matching in
the paper's pipeline (Section 3.6, "GPU MAGSAC++": 1,500 minimal-sample
hypotheses solved in one batch and scored by soft marginalisation over the
noise scale).  Only tests/ and the benchmark's CPU baseline use it.

The paper names the estimator and gives no formulas; the readings taken here
(identical on the GPU) are:

* Model: a planar homography H mapping points of image a to image b, found
  in normalised coordinates (each point set moved to zero mean and scaled to
  mean distance sqrt(2) from it, over all correspondences) with h33 = 1.
* Hypotheses: K minimal samples of 4 correspondences.  The random numbers are
  inputs: sample k takes correspondences floor(u[k, j] * N), j = 0..3, for
  u[k, j] in [0, 1).  A sample with a repeated index or a singular 8 x 8
  system (a pivot below 1e-12 of the largest entry) gives no hypothesis.
* Residual: r = |pi(H a) - b| in pixels of image b; a point mapped to or
  behind the line at infinity (projective denominator <= 0) is an outlier.
* Soft marginalisation: for a noise scale sigma the residual of an inlier is
  Rayleigh distributed (2-D Gaussian error), truncated at its 0.99 quantile
  tau * sigma, tau = sqrt(2 ln 100); with sigma uniform on (0, sigma_max] the
  marginal likelihood of residual r is
      w(r) = (1 / sigma_max) * integral_{r / tau}^{sigma_max} (r / s^2) exp(-r^2 / (2 s^2)) ds
           = sqrt(pi / 2) / sigma_max * (erf(tau / sqrt 2) - erf(r / (sqrt 2 sigma_max)))
  for r < tau * sigma_max and 0 beyond.  A hypothesis scores Q = sum_i w(r_i);
  the best is the largest Q (smallest index among equals).
* Refinement (iteratively reweighted least squares): each step solves the
  weighted normal equations sum_i w(r_i) A_i^T A_i h = sum_i w(r_i) A_i^T b_i of
  the DLT rows in normalised coordinates, w from the current model's
  residuals; a step is kept only if it raises Q, and refinement stops at the
  first step that does not, or after `refine_iters` steps.
* Output: H (h33 = 1, image coordinates), Q, the number of correspondences
  with w > 0, the index of the best hypothesis.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

TAU = math.sqrt(2.0 * math.log(100.0))
PIVOT_EPS = 1e-12


def marginal_weight(r, sigma_max: float):
    """w(r): the closed form of the sigma-marginalised truncated Rayleigh
    likelihood (module docstring)."""
    r = np.asarray(r, dtype=np.float64)
    from scipy.special import erf
    w = math.sqrt(math.pi / 2.0) / sigma_max * (erf(TAU / math.sqrt(2.0))
                                                - erf(r / (math.sqrt(2.0) * sigma_max)))
    return np.where(np.isfinite(r) & (r < TAU * sigma_max), w, 0.0)


def normaliser(pts: np.ndarray) -> np.ndarray:
    """3 x 3 similarity moving the points to zero mean and mean distance sqrt(2)."""
    c = pts.mean(axis=0)
    d = np.mean(np.sqrt(np.sum((pts - c) ** 2, axis=1)))
    s = math.sqrt(2.0) / d if d > 0 else 1.0
    return np.array([[s, 0.0, -s * c[0]], [0.0, s, -s * c[1]], [0.0, 0.0, 1.0]])


def apply(H: np.ndarray, pts: np.ndarray):
    """Projected points and the projective denominators."""
    x = pts[:, 0] * H[0, 0] + pts[:, 1] * H[0, 1] + H[0, 2]
    y = pts[:, 0] * H[1, 0] + pts[:, 1] * H[1, 1] + H[1, 2]
    w = pts[:, 0] * H[2, 0] + pts[:, 1] * H[2, 1] + H[2, 2]
    return np.stack([x / w, y / w], axis=1), w


def residuals(H: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    proj, den = apply(H, a)
    r = np.sqrt(np.sum((proj - b) ** 2, axis=1))
    return np.where(den > 0, r, np.inf)


def dlt_rows(a: np.ndarray, b: np.ndarray):
    """Rows of the DLT system A h = rhs for h = (h11..h32), h33 = 1."""
    n = len(a)
    A = np.zeros((2 * n, 8))
    rhs = np.zeros(2 * n)
    x, y, u, v = a[:, 0], a[:, 1], b[:, 0], b[:, 1]
    A[0::2, 0], A[0::2, 1], A[0::2, 2] = x, y, 1.0
    A[0::2, 6], A[0::2, 7] = -u * x, -u * y
    A[1::2, 3], A[1::2, 4], A[1::2, 5] = x, y, 1.0
    A[1::2, 6], A[1::2, 7] = -v * x, -v * y
    rhs[0::2], rhs[1::2] = u, v
    return A, rhs


def solve8(M: np.ndarray, rhs: np.ndarray):
    """h of M h = rhs by Gaussian elimination with partial pivoting, or None
    when a pivot falls below PIVOT_EPS of the largest entry of M."""
    M = M.astype(np.float64).copy()
    rhs = rhs.astype(np.float64).copy()
    scale = np.max(np.abs(M))
    if not scale > 0:
        return None
    n = len(rhs)
    for col in range(n):
        piv = col + int(np.argmax(np.abs(M[col:, col])))
        if abs(M[piv, col]) < PIVOT_EPS * scale:
            return None
        if piv != col:
            M[[col, piv]] = M[[piv, col]]
            rhs[[col, piv]] = rhs[[piv, col]]
        for row in range(col + 1, n):
            f = M[row, col] / M[col, col]
            M[row, col:] -= f * M[col, col:]
            rhs[row] -= f * rhs[col]
    h = np.zeros(n)
    for row in range(n - 1, -1, -1):
        h[row] = (rhs[row] - M[row, row + 1:] @ h[row + 1:]) / M[row, row]
    return h


def h_matrix(h8: np.ndarray) -> np.ndarray:
    return np.append(h8, 1.0).reshape(3, 3)


def denormalise(Hn: np.ndarray, Ta: np.ndarray, Tb: np.ndarray) -> np.ndarray:
    H = np.linalg.inv(Tb) @ Hn @ Ta
    return H / H[2, 2]


@dataclass
class VerifyResult:
    H: np.ndarray            # 3 x 3, h33 = 1 (NaN when no hypothesis)
    score: float
    n_inliers: int
    best: int                # index of the best hypothesis, -1 if none
    scores: np.ndarray       # [K] score of every hypothesis (-inf: none)
    steps_kept: int          # refinement steps kept


def sample_indices(u: np.ndarray, n: int) -> np.ndarray:
    return np.minimum(np.floor(np.asarray(u, dtype=np.float64) * n).astype(np.int64), n - 1)


def verify(a: np.ndarray, b: np.ndarray, u: np.ndarray, sigma_max: float = 2.0,
           refine_iters: int = 5) -> VerifyResult:
    """Homography verification of correspondences a[i] <-> b[i] (N x 2, pixels)
    with the minimal samples drawn from u (K x 4 numbers in [0, 1))."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, 2)
    b = np.asarray(b, dtype=np.float64).reshape(-1, 2)
    n = len(a)
    K = len(u)
    nan = np.full((3, 3), np.nan)
    if n < 4:
        return VerifyResult(nan, 0.0, 0, -1, np.full(K, -np.inf), 0)
    Ta, Tb = normaliser(a), normaliser(b)
    an = (np.c_[a, np.ones(n)] @ Ta.T)[:, :2]
    bn = (np.c_[b, np.ones(n)] @ Tb.T)[:, :2]
    idx = sample_indices(u, n)
    scores = np.full(K, -np.inf)
    models = [None] * K
    for k in range(K):
        s = idx[k]
        if len(set(s.tolist())) < 4:
            continue
        A, rhs = dlt_rows(an[s], bn[s])
        h = solve8(A, rhs)
        if h is None:
            continue
        H = denormalise(h_matrix(h), Ta, Tb)
        if not np.all(np.isfinite(H)):
            continue
        models[k] = H
        scores[k] = float(np.sum(marginal_weight(residuals(H, a, b), sigma_max)))
    if not np.any(np.isfinite(scores)):
        return VerifyResult(nan, 0.0, 0, -1, scores, 0)
    best = int(np.argmax(scores))           # first of the largest
    H, Q = models[best], scores[best]
    kept = 0
    for _ in range(refine_iters):
        w = marginal_weight(residuals(H, a, b), sigma_max)
        A, rhs = dlt_rows(an, bn)
        ww = np.repeat(w, 2)
        h = solve8(A.T @ (ww[:, None] * A), A.T @ (ww * rhs))
        if h is None:
            break
        H2 = denormalise(h_matrix(h), Ta, Tb)
        if not np.all(np.isfinite(H2)):
            break
        Q2 = float(np.sum(marginal_weight(residuals(H2, a, b), sigma_max)))
        if not Q2 > Q:
            break
        H, Q = H2, Q2
        kept += 1
    n_in = int(np.sum(marginal_weight(residuals(H, a, b), sigma_max) > 0))
    return VerifyResult(H, Q, n_in, best, scores, kept)

"""Reference symmetric ratio-test matcher (test infrastructure only).

Plain FP64 NumPy statement of the matching step that follows extraction in
the paper's pipeline (Section 3.4, "Descriptor Matching", backend (1)): a
similarity matrix of the two descriptor sets computed from fp16 inputs, a
nearest-neighbour ratio test, and mutual-consistency filtering.  It is slow
and obviously correct; only tests/, the smoke entry point and the benchmark's
CPU baseline use it, never the library.

What the paper leaves open, and the reading taken here (identical on the GPU):

* Similarity: s_ij = <a_i, b_j> of the descriptors rounded to fp16 (round to
  nearest even), the products summed without further rounding (the kernel
  accumulates in fp32).  The paper's matmul runs "at fp16"; its result is
  read here as the fp32 accumulator, not rounded to fp16 again (which would
  make most decisions ties).
* Distance: descriptors are unit L2 vectors (plain SIFT and RootSIFT both end
  L2-normalised), so the squared Euclidean distance is D = max(2 - 2 s, 0).
* Ratio test (Lowe's): the nearest neighbour passes when D1 < r^2 D2, D2 the
  second-nearest neighbour's squared distance; r = 0.8 by default.  With a
  single candidate there is no second neighbour and D2 is taken as 4 (the
  largest distance between unit vectors).
* Symmetric: the test runs both ways (a's nearest in b and b's nearest in a)
  and a pair is kept only when each is the other's nearest neighbour (mutual)
  and both ratio tests pass.
* Ties: the nearest neighbour is the candidate of largest similarity, the
  smallest index among equals; equal best similarities make D1 = D2, so the
  ratio test then fails whatever the index.
* Output: kept pairs (i, j) in ascending i, with s_ij and sqrt(D).

Decisions are taken on the fp32 value of every similarity (the precision of
the kernel's accumulator).  Each is logged with its margin in similarity
units; a row is *decisive* when every margin that decides it exceeds the fp32
accumulation error of a 128-term dot product of unit vectors (see TOL).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Largest |s_fp32 accumulation - s_exact| for 128 products of unit vectors:
# gamma_128 * sum |a_k b_k| <= 128 * 2^-24 * 1 (plus the fp16-rounded norms'
# 1e-3 slack), rounded up.  Margins at or below it are marginal.
TOL = 2e-5
NO_SECOND_D = 4.0


def round_fp16(desc: np.ndarray) -> np.ndarray:
    """Descriptors as the matcher sees them: fp16 (RNE) values, as float64."""
    return np.asarray(desc, dtype=np.float32).astype(np.float16).astype(np.float64)


def similarity(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Exact s_ij = <fp16(a_i), fp16(b_j)> (products of fp16 values are exact
    in fp64 and 128 of them sum with error far below fp32's)."""
    return round_fp16(a) @ round_fp16(b).T


def sq_dist(s) -> np.ndarray:
    return np.maximum(2.0 - 2.0 * np.asarray(s, dtype=np.float64), 0.0)


def top2(s_rows: np.ndarray):
    """Per row of s_rows (float32 values): (best index, best value, second
    value); the smallest index wins among equal values; with one column the
    second value is NaN (no second neighbour)."""
    n, m = s_rows.shape
    best = np.zeros(n, dtype=np.int64)
    s1 = np.full(n, np.nan)
    s2 = np.full(n, np.nan)
    if m == 0:
        return np.full(n, -1, dtype=np.int64), s1, s2
    best = np.argmax(s_rows, axis=1)          # first occurrence of the maximum
    s1 = s_rows[np.arange(n), best].astype(np.float64)
    if m > 1:
        rest = s_rows.astype(np.float64).copy()
        rest[np.arange(n), best] = -np.inf
        s2 = rest.max(axis=1)
    return best, s1, s2


def ratio_sq(ratio: float) -> np.float32:
    """r^2 as the kernel holds it: the ratio is an fp32 setting, squared in
    double precision and rounded to fp32."""
    rf = float(np.float32(ratio))
    return np.float32(rf * rf)


def ratio_ok(s1, s2, ratio: float):
    """Ratio test in fp32 as the kernel takes it: D1 < fp32(r^2) * D2."""
    r2 = ratio_sq(ratio)
    d1 = np.maximum(np.float32(2.0) - np.float32(2.0) * np.float32(s1), np.float32(0.0))
    d2 = (np.float32(NO_SECOND_D) if np.isnan(s2)
          else np.maximum(np.float32(2.0) - np.float32(2.0) * np.float32(s2), np.float32(0.0)))
    return bool(d1 < np.float32(r2 * d2)), float(r2) * float(d2) - float(d1)


@dataclass
class MatchResult:
    pairs: np.ndarray                 # int64 [K, 2] (i, j), ascending i
    sim: np.ndarray                   # float64 [K] exact similarities
    dist: np.ndarray                  # float64 [K] sqrt(D)
    decisive: np.ndarray              # bool [n_a] every deciding margin > TOL
    row_best: np.ndarray              # int64 [n_a] nearest j (-1 if none)
    log: list = field(default_factory=list)   # per row: dict of margins


def match(a: np.ndarray, b: np.ndarray, ratio: float = 0.8) -> MatchResult:
    """Symmetric ratio-test matching of descriptor sets a [n_a, 128] and
    b [n_b, 128] (Section 3.4, backend (1), with the readings above)."""
    a = np.asarray(a, dtype=np.float32).reshape(-1, 128)
    b = np.asarray(b, dtype=np.float32).reshape(-1, 128)
    na, nb = len(a), len(b)
    s_exact = similarity(a, b) if na and nb else np.zeros((na, nb))
    s32 = s_exact.astype(np.float32)          # the decisions' precision
    rb, rs1, rs2 = top2(s32)                  # a_i's nearest in b
    cb, cs1, cs2 = top2(s32.T)                # b_j's nearest in a
    pairs, sims, dists, log = [], [], [], []
    decisive = np.zeros(na, dtype=bool)
    for i in range(na):
        if nb == 0:
            log.append({})
            continue
        j = int(rb[i])
        row_gap = np.inf if np.isnan(rs2[i]) else float(rs1[i] - rs2[i])
        ok_r, m_r = ratio_ok(rs1[i], rs2[i], ratio)
        mutual = int(cb[j]) == i
        col_gap = np.inf if np.isnan(cs2[j]) else float(cs1[j] - cs2[j])
        ok_c, m_c = ratio_ok(cs1[j], cs2[j], ratio)
        # the exact value sits within TOL of what either side computes: a gap
        # or ratio margin above the tolerance fixes the decision
        margins = {"row_gap": row_gap, "ratio_row": abs(m_r) / 4.0,
                   "col_gap": col_gap, "ratio_col": abs(m_c) / 4.0}
        decisive[i] = all(v > TOL for v in margins.values())
        log.append(dict(margins, j=j, mutual=mutual, ok_r=ok_r, ok_c=ok_c))
        if mutual and ok_r and ok_c:
            pairs.append((i, j))
            sims.append(s_exact[i, j])
            dists.append(np.sqrt(sq_dist(s_exact[i, j])))
    return MatchResult(np.array(pairs, dtype=np.int64).reshape(-1, 2),
                       np.array(sims, dtype=np.float64), np.array(dists, dtype=np.float64),
                       decisive, rb.astype(np.int64) if nb else np.full(na, -1), log)


def match_bruteforce(a, b, ratio: float = 0.8):
    """The same decisions by explicit loops (tiny inputs only): used to pin
    the vectorised form."""
    a16, b16 = round_fp16(a), round_fp16(b)
    na, nb = len(a16), len(b16)
    s = [[np.float32(sum(float(a16[i, k]) * float(b16[j, k]) for k in range(a16.shape[1])))
          for j in range(nb)] for i in range(na)]

    def nn(values):
        best = 0
        for idx in range(1, len(values)):
            if values[idx] > values[best]:
                best = idx
        rest = [v for idx, v in enumerate(values) if idx != best]
        return best, values[best], (max(rest) if rest else None)

    out = []
    for i in range(na):
        if nb == 0:
            break
        j, s1, s2 = nn(s[i])
        ci, c1, c2 = nn([s[q][j] for q in range(na)])
        ok_r = ratio_ok(s1, np.nan if s2 is None else s2, ratio)[0]
        ok_c = ratio_ok(c1, np.nan if c2 is None else c2, ratio)[0]
        if ci == i and ok_r and ok_c:
            out.append((i, j))
    return out

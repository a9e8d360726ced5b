"""Keypoint/descriptor comparison between an extraction result and the oracle.

Decision rule: an oracle candidate is *decisive* when every margin it logged
(pre-gate, extremum, Newton-step rounding, contrast, edge, orientation window
radius, orientation peaks) exceeds ``MARGIN``; otherwise it is *marginal*
and either outcome is accepted.  For decisive candidates the result under
test must reproduce the oracle's accept/reject decision, the integer
(octave, layer, row, col), the number of orientations, and the values within
the tolerances below.  Every keypoint under test must come from an oracle
candidate, or from a pixel whose candidate test is itself marginal.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MARGIN = 1e-4
TOL_XY = 1e-3          # input-image pixels
TOL_ANGLE = 0.1        # degrees, circular
TOL_DESC = 2e-3        # max-abs on the normalised descriptor
TOL_REL = 1e-4         # sigma and response, relative

MARGIN_KEYS = ("m_pre", "m_ext", "m_move", "m_con", "m_edge", "m_peak", "m_rad")


def is_decisive(entry: dict, margin: float = MARGIN) -> bool:
    return all(entry.get(k, math.inf) > margin for k in MARGIN_KEYS)


def angle_diff(a, b):
    d = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)) % 360.0
    return np.minimum(d, 360.0 - d)


@dataclass
class Report:
    decisive_ok: int = 0
    decisive_rejected: int = 0
    marginal: int = 0
    extra_marginal: int = 0
    checked_keypoints: int = 0
    max_err_xy: float = 0.0
    max_err_angle: float = 0.0
    max_err_desc: float = 0.0
    max_err_rel: float = 0.0
    mismatches: list = field(default_factory=list)

    @property
    def ok(self) -> bool:
        return not self.mismatches

    def summary(self) -> str:
        return (f"decisive_ok={self.decisive_ok} decisive_rejected={self.decisive_rejected} "
                f"marginal={self.marginal} extra_marginal={self.extra_marginal} "
                f"checked_kp={self.checked_keypoints} max_xy={self.max_err_xy:.3g} "
                f"max_angle={self.max_err_angle:.3g} max_desc={self.max_err_desc:.3g} "
                f"max_rel={self.max_err_rel:.3g} mismatches={len(self.mismatches)}")


def group_by_source(kps) -> dict:
    """{(octave, src_layer, src_iy, src_ix): [row indices in order]}"""
    groups: dict = {}
    for k in range(len(kps)):
        key = (int(kps["octave"][k]), int(kps["src_layer"][k]),
               int(kps["src_iy"][k]), int(kps["src_ix"][k]))
        groups.setdefault(key, []).append(k)
    return groups


def source_keys(kps) -> list:
    """(octave, src_layer, src_iy, src_ix) of every keypoint, in output order."""
    return [(int(kps["octave"][k]), int(kps["src_layer"][k]), int(kps["src_iy"][k]),
             int(kps["src_ix"][k])) for k in range(len(kps))]


def check_order(oracle_result, kps, rep: Report, margin: float = MARGIN, before=None):
    """Canonical order: keypoints come by ascending source detection (octave,
    layer, row, column), and, over the decisive detections, the sequence of
    source keys (one per orientation) equals the oracle's.  ``before``: only
    keys below it take part (the cut of a capped output)."""
    keys = source_keys(kps)
    for a, b in zip(keys, keys[1:]):
        if b < a:
            rep.mismatches.append((b, f"out of canonical order after {a}"))
            break
    decisive = {(e["o"], e["i0"], e["r0"], e["c0"]): e for e in oracle_result.log
                if is_decisive(e, margin)}
    want = []
    for key, e in decisive.items():
        if before is not None and not key < before:
            continue
        if e["status"] == "ok":
            want += [key] * len(e["angles"])
    got = [k for k in keys if k in decisive and (before is None or k < before)]
    if got != want:
        first = next((j for j, (a, b) in enumerate(zip(got, want)) if a != b),
                     min(len(got), len(want)))
        rep.mismatches.append((got[first] if first < len(got) else None,
                               f"decisive key sequence differs from the oracle's at position "
                               f"{first} ({len(got)} vs {len(want)} keys)"))


def compare(oracle_result, kps, desc, params, oracle_mod, margin: float = MARGIN,
            sample: set | None = None, before=None, tol: dict | None = None) -> Report:
    """Compare keypoints ``kps`` (structured array with the oracle's field
    names) and descriptors ``desc`` with ``oracle_result``, including their
    canonical order.

    ``sample``: optional set of candidate keys to restrict the check to (for
    large inputs where the oracle describes only some candidates).
    ``before``: only source keys below this one are compared (a capped output
    is the prefix of the canonical sequence up to its cut; see
    ``compare_capped``).  Without it the check assumes no cap was hit.
    ``tol``: overrides of the value tolerances (keys xy, angle, desc, rel)."""
    rep = Report()
    t = dict(xy=TOL_XY, angle=TOL_ANGLE, desc=TOL_DESC, rel=TOL_REL)
    t.update(tol or {})
    got = group_by_source(kps)
    by_key = {(e["o"], e["i0"], e["r0"], e["c0"]): e for e in oracle_result.log}
    octs = {oc.o: oc for oc in oracle_result.octaves}
    if sample is None:
        check_order(oracle_result, kps, rep, margin, before)
    for key, e in by_key.items():
        if sample is not None and key not in sample:
            continue
        if before is not None and not key < before:
            continue
        if not is_decisive(e, margin):
            rep.marginal += 1
            continue
        rows = got.get(key, [])
        if e["status"] != "ok":
            rep.decisive_rejected += 1
            if rows:
                rep.mismatches.append((key, f"oracle rejected ({e['status']}) but result has "
                                            f"{len(rows)} keypoints"))
            continue
        rep.decisive_ok += 1
        angles = e["angles"]
        if len(rows) != len(angles):
            rep.mismatches.append((key, f"orientation count {len(rows)} != oracle {len(angles)}"))
            continue
        for k, row in enumerate(rows):
            kp = kps[row]
            if (int(kp["layer"]), int(kp["iy"]), int(kp["ix"])) != (e["i"], e["r"], e["c"]):
                rep.mismatches.append((key, f"integer position {(int(kp['layer']), int(kp['iy']), int(kp['ix']))}"
                                            f" != oracle {(e['i'], e['r'], e['c'])}"))
                continue
            exy = max(abs(float(kp["x"]) - e["x"]), abs(float(kp["y"]) - e["y"]))
            ea = float(angle_diff(kp["angle"], angles[k]))
            ed = float(np.max(np.abs(np.asarray(desc[row], dtype=np.float64) - e["desc"][k])))
            er = max(abs(float(kp["sigma"]) - e["sigma"]) / e["sigma"],
                     abs(float(kp["response"]) - e["response"]) / e["response"])
            rep.max_err_xy = max(rep.max_err_xy, exy)
            rep.max_err_angle = max(rep.max_err_angle, ea)
            rep.max_err_desc = max(rep.max_err_desc, ed)
            rep.max_err_rel = max(rep.max_err_rel, er)
            rep.checked_keypoints += 1
            bad = []
            if exy > t["xy"]:
                bad.append(f"xy err {exy:.3g}")
            if ea > t["angle"]:
                bad.append(f"angle err {ea:.3g}")
            if ed > t["desc"]:
                bad.append(f"desc err {ed:.3g}")
            if er > t["rel"]:
                bad.append(f"sigma/response rel err {er:.3g}")
            if bad:
                rep.mismatches.append((key, ", ".join(bad)))
    # keypoints from pixels the oracle did not take as candidates
    for key, rows in got.items():
        if key in by_key:
            continue
        if sample is not None and key not in sample:
            continue
        if before is not None and not key < before:
            continue
        o, i, r, c = key
        oc = octs.get(o)
        if oc is None:
            rep.mismatches.append((key, "keypoint from an octave the oracle does not have"))
            continue
        m = oracle_mod.pixel_margins(oc.D, i, r, c, params)
        if min(m["m_pre"], m["m_ext"]) <= margin:
            rep.extra_marginal += 1
        else:
            rep.mismatches.append((key, f"not an oracle candidate (margins {m})"))
    return rep


def compare_capped(oracle_full, kps, desc, params, oracle_mod, cap: int,
                   margin: float = MARGIN) -> Report:
    """A keypoint-capped output against the uncapped oracle: the output must be
    the first ``cap`` keypoints of the canonical sequence.  Every source key
    below the output's last one is compared in full (values, orientation
    counts, order).  When no marginal detection precedes the cut on either
    side, the output's key sequence must equal the oracle's first ``cap``
    keys exactly (so both cut at the same keypoint)."""
    keys = source_keys(kps)
    if not keys:
        rep = Report()
        rep.mismatches.append((None, "capped output is empty"))
        return rep
    cut = keys[-1]
    rep = compare(oracle_full, kps, desc, params, oracle_mod, margin, before=cut)
    if len(kps) > cap:
        rep.mismatches.append((cut, f"{len(kps)} keypoints under a cap of {cap}"))
    full_keys = []
    for e in oracle_full.log:
        if e["status"] == "ok":
            full_keys += [(e["o"], e["i0"], e["r0"], e["c0"])] * len(e["angles"])
    o_cap = full_keys[:cap]
    limit = max(cut, o_cap[-1]) if o_cap else cut
    marginal_before = any(not is_decisive(e, margin) and (e["o"], e["i0"], e["r0"], e["c0"]) <= limit
                          for e in oracle_full.log)
    if not marginal_before and rep.extra_marginal == 0 and keys != o_cap:
        rep.mismatches.append((cut, f"capped key sequence differs from the oracle's first {cap}"))
    return rep

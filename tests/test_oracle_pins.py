"""Pins of the FP64 oracle against closed forms, library routines, brute force
and invariants (CPU only)."""
import json
import math
from pathlib import Path

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from oracle import sift_oracle as so

GOLDEN = Path(__file__).parent / "golden"


def p_default(**kw):
    p = so.Params()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# ---------------------------------------------------------------- P1 taps

def test_taps_sum_symmetry_and_radius():
    for sigma in (0.7, 1.2263, 1.5199, 2.4525, 3.09, 5.5):
        r, g = so.gaussian_taps(sigma)
        assert r == math.ceil(4 * sigma)
        assert len(g) == 2 * r + 1
        assert abs(g.sum() - 1.0) < 1e-15
        assert np.array_equal(g, g[::-1])
        assert np.all(np.diff(g[: r + 1]) > 0)


def test_level_sigmas_compose_to_the_scale_schedule():
    """Applied blurs add in quadrature to sigma0 * k^i (k = 2^(1/s)), starting
    from the assumed input blur (0.5, doubled by the 2x upsample)."""
    for up in (0, 1):
        p = p_default(upsample=up)
        init, incs = so.level_sigmas(p)
        assumed = 0.5 * (2 if up else 1)
        total2 = assumed ** 2 + init ** 2
        assert abs(total2 - 1.6 ** 2) < 1e-12
        for i, s in enumerate(incs, start=1):
            total2 += s * s
            assert abs(math.sqrt(total2) - 1.6 * 2 ** (i / 3)) < 1e-12
    # radii of the default schedule: ceil(4 sigma)
    _, incs = so.level_sigmas(p_default())
    assert [so.gaussian_taps(s)[0] for s in incs] == [5, 7, 8, 10, 13]


def test_golden_constants_used_by_the_oracle():
    """Constants the paper states (section 3.2) as stored in the golden file."""
    c = json.loads((GOLDEN / "paper_constants.json").read_text())
    p = so.Params()
    assert p.ori_bins == c["orientation_bins"]["value"]
    assert p.refine_iters == c["max_refinement_iterations"]["value"]
    h = np.zeros(p.ori_bins)
    h[5] = 1.0
    angles, _ = so.orientation_peaks(h, p)
    # one smoothing pass with the stated kernel: the neighbours receive 1/4
    sm = 0.25 * np.roll(h, 1) + 0.5 * h + 0.25 * np.roll(h, -1)
    assert np.allclose(sm[4:7], c["orientation_smoothing"]["value"])
    assert angles == [50.0]
    paper_dsp = c["dsp_scales_paper"]["value"]
    assert np.allclose(paper_dsp, [0.5, 1 / math.sqrt(2), 1.0, math.sqrt(2), 2.0])
    r, _ = so.gaussian_taps(2.0)
    assert r == math.ceil(c["gaussian_truncation_sigmas"]["value"] * 2.0)


# ---------------------------------------------------------------- P2 blur

@pytest.mark.parametrize("shape,sigma", [((23, 31), 1.3), ((9, 7), 2.2), ((5, 6), 1.9)])
def test_blur_equals_scipy_mirror_and_direct_2d(shape, sigma):
    rng = np.random.default_rng(1)
    img = rng.random(shape)
    r, g = so.gaussian_taps(sigma)
    ours = so.gaussian_blur(img, sigma)
    # SciPy's 'mirror' mode is reflect-101 with repeated reflection
    ref = ndi.correlate1d(ndi.correlate1d(img, g, axis=1, mode="mirror"), g, axis=0, mode="mirror")
    assert np.max(np.abs(ours - ref)) < 1e-15 * 20
    # direct 2-D correlation with outer(g, g), indices mirrored by hand
    h, w = shape
    k2 = np.outer(g, g)
    direct = np.zeros_like(img)
    for y in range(h):
        for x in range(w):
            acc = 0.0
            for dy in range(-r, r + 1):
                yy = so.mirror_index(y + dy, h)
                for dx in range(-r, r + 1):
                    acc += k2[dy + r, dx + r] * img[yy, so.mirror_index(x + dx, w)]
            direct[y, x] = acc
    assert np.max(np.abs(ours - direct)) < 1e-14


def test_mirror_index_examples():
    n = 5
    assert list(so.mirror_index(np.arange(-6, 11), n)) == \
        [2, 3, 4, 3, 2, 1, 0, 1, 2, 3, 4, 3, 2, 1, 0, 1, 2]
    assert list(so.mirror_index(np.array([-3, 0, 4]), 1)) == [0, 0, 0]


def test_upsample_matches_scipy_linear_interpolation():
    rng = np.random.default_rng(2)
    img = rng.random((7, 9))
    up = so.upsample2x(img)
    yy, xx = np.mgrid[0:14, 0:18] / 2.0
    ref = ndi.map_coordinates(img, [yy, xx], order=1, mode="nearest")
    assert np.max(np.abs(up - ref)) < 1e-15
    assert np.array_equal(up[0::2, 0::2], img)


# ---------------------------------------------------------------- P3 / P4 invariants

def test_constant_image_has_flat_pyramid_and_no_keypoints():
    img = np.full((64, 80), 0.37, dtype=np.float32)
    p = p_default(n_octaves=3)
    octs = so.scale_space(img, p)
    for oc in octs:
        assert np.max(np.abs(oc.L - np.float64(np.float32(0.37)))) < 1e-14
        assert np.max(np.abs(oc.D)) < 1e-14
    res = oracle.sift(img, p)
    assert len(res.keypoints) == 0 and len(res.log) == 0


def test_ramp_is_preserved_away_from_borders():
    h, w = 90, 100
    yy, xx = np.mgrid[0:h, 0:w]
    img = (0.2 + 0.003 * xx + 0.002 * yy)
    out = so.gaussian_blur(img, 2.4525)
    r = 10
    assert np.max(np.abs(out[r:-r, r:-r] - img[r:-r, r:-r])) < 1e-13
    p = p_default(n_octaves=2)
    octs = so.scale_space(img.astype(np.float32), p)
    # interior DoG vanishes (the ramp survives every blur of the chain)
    m = 40
    assert np.max(np.abs(octs[0].D[:, m:-m, m:-m])) < 1e-6


# ---------------------------------------------------------------- P5 blob scale

def closed_form_centre_dog(amp, sb, sigma_total_sq_minus_in):
    return amp * sb * sb / (sb * sb + sigma_total_sq_minus_in)


@pytest.mark.parametrize("sb", [3.0, 4.0, 6.0])
def test_gaussian_blob_detected_at_its_centre_and_scale(sb):
    n = 129
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    amp = 0.3
    img = 0.5 + amp * np.exp(-((xx - 64) ** 2 + (yy - 64) ** 2) / (2 * sb * sb))
    p = p_default(n_octaves=3)
    res = oracle.sift(img.astype(np.float32), p, describe=False)
    ok = [e for e in res.log if e["status"] == "ok"]
    at = [e for e in ok if abs(e["x"] - 64) < 1e-6 and abs(e["y"] - 64) < 1e-6]
    assert at, f"no keypoint at the blob centre ({len(ok)} keypoints)"
    e = at[0]
    # by symmetry the sub-pixel offset is zero in x and y
    assert abs(e["xhat"][0]) < 1e-9 and abs(e["xhat"][1]) < 1e-9
    # scale offset: the same 3-point fit on the continuous-blur centre DoG
    o, i = e["o"], e["i"]
    s = p.n_scales
    total = [p.sigma0 * 2 ** o * 2 ** (j / s) for j in range(i - 1, i + 3)]
    Lc = [0.5 + closed_form_centre_dog(amp, sb, t * t - p.sigma_in ** 2) for t in total]
    Dc = np.diff(Lc)
    xs_pred = -0.5 * (Dc[2] - Dc[0]) / (Dc[2] + Dc[0] - 2 * Dc[1])
    assert abs(e["xhat"][2] - xs_pred) < 2e-2
    # the detected scale brackets the blob's characteristic DoG scale
    sig = p.sigma0 * 2 ** o * 2 ** ((i + e["xhat"][2]) / s)
    assert 0.6 * sb < sig < 1.3 * sb


# ---------------------------------------------------------------- P6 extrema

def test_candidate_mask_equals_brute_force():
    rng = np.random.default_rng(3)
    D = rng.normal(0, 0.02, (5, 20, 23))
    D[2, 10, 11] = 0.2
    D[1, 6, 7] = -0.3
    p = p_default(border=2)
    thr = p.prefilter_ratio * p.contrast_threshold
    for i in (1, 2, 3):
        mask = so.candidate_mask(D, i, p)
        brute = np.zeros_like(mask)
        for r in range(p.border, 20 - p.border):
            for c in range(p.border, 23 - p.border):
                v = D[i, r, c]
                if abs(v) <= thr:
                    continue
                nbs = [D[i + a, r + b, c + d] for a in (-1, 0, 1) for b in (-1, 0, 1)
                       for d in (-1, 0, 1) if (a, b, d) != (0, 0, 0)]
                if all(v > x for x in nbs) or all(v < x for x in nbs):
                    brute[r, c] = True
        assert np.array_equal(mask, brute)
    assert so.candidate_mask(D, 2, p)[10, 11] and so.candidate_mask(D, 1, p)[6, 7]


# ---------------------------------------------------------------- P7 / P8 refinement

def test_cramer_matches_numpy_solve():
    rng = np.random.default_rng(4)
    for _ in range(50):
        H = rng.normal(size=(3, 3))
        H = H + H.T
        b = rng.normal(size=3)
        x, det = so.cramer_solve(H, b)
        ref = np.linalg.solve(H, b)
        assert np.max(np.abs(x - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))
        assert abs(det - np.linalg.det(H)) <= 1e-10 * max(1.0, abs(det))


def quadratic_octave(centre, hess, peak=-0.05, shape=(5, 31, 33)):
    """DoG stack sampled from q(p) = peak + 1/2 (p - centre)^T H (p - centre),
    p = (x, y, s): central differences are exact on it."""
    s_, h, w = shape
    ii, rr, cc = np.meshgrid(np.arange(s_), np.arange(h), np.arange(w), indexing="ij")
    d = np.stack([cc - centre[0], rr - centre[1], ii - centre[2]], axis=-1).astype(np.float64)
    q = peak + 0.5 * np.einsum("...a,ab,...b->...", d, np.asarray(hess, dtype=np.float64), d)
    L = np.zeros((s_ + 1, h, w))
    L[1:] = np.cumsum(q, axis=0)
    return so.Octave(0, L, q)


def test_refine_recovers_exact_extremum_of_a_quadratic():
    H = np.array([[0.02, 0.003, 0.001], [0.003, 0.03, 0.002], [0.001, 0.002, 0.05]])
    centre = (15.7, 13.2, 2.3)        # 0.7 from the start column: one step needed
    oc = quadratic_octave(centre, H, peak=-0.05)
    p = p_default(border=3)
    res = so.refine(oc, 2, 13, 15, p)
    assert res["status"] == "ok"
    assert (res["c"], res["r"], res["i"]) == (16, 13, 2)
    assert np.allclose([res["c"] + res["xhat"][0], res["r"] + res["xhat"][1],
                        res["i"] + res["xhat"][2]], centre, atol=1e-10)
    assert abs(res["contrast"] - (-0.05)) < 1e-12
    assert res["sigma_oct"] == pytest.approx(1.6 * 2 ** (2.3 / 3), rel=1e-12)


def test_refine_rejects_far_and_unconverged_steps():
    H = np.diag([0.02, 0.02, 0.04])
    oc = quadratic_octave((30.9, 13.0, 2.0), H)      # leaves the frame
    assert so.refine(oc, 2, 13, 26, p_default(border=3))["status"] == "bounds"
    p = p_default(border=3, refine_iters=1)
    oc = quadratic_octave((16.8, 13.0, 2.0), H)      # needs a second iteration
    assert so.refine(oc, 2, 13, 15, p)["status"] == "no_converge"


@pytest.mark.parametrize("ratio,keep", [(5.0, True), (9.9, True), (10.1, False), (20.0, False)])
def test_edge_test_threshold_on_principal_curvature_ratio(ratio, keep):
    a = 0.01
    H = np.diag([a, a * ratio, 0.05])
    oc = quadratic_octave((15.0, 13.0, 2.0), H, peak=-0.05)
    res = so.refine(oc, 2, 13, 15, p_default(border=3))
    assert (res["status"] == "ok") == keep
    if not keep:
        assert res["status"] == "edge"


def test_contrast_test():
    H = np.diag([0.02, 0.02, 0.04])
    p = p_default(border=3)
    low = quadratic_octave((15.0, 13.0, 2.0), H, peak=-0.9 * p.contrast_threshold)
    assert so.refine(low, 2, 13, 15, p)["status"] == "contrast"
    high = quadratic_octave((15.0, 13.0, 2.0), H, peak=-1.1 * p.contrast_threshold)
    assert so.refine(high, 2, 13, 15, p)["status"] == "ok"


# ---------------------------------------------------------------- P9 orientation

@pytest.mark.parametrize("phi_deg", [0.0, 30.0, 93.0, 181.0, 237.5, 304.0, 359.0])
def test_orientation_of_a_ramp_follows_the_soft_bin_closed_form(phi_deg):
    phi = math.radians(phi_deg)
    n = 61
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    L = math.cos(phi) * xx + math.sin(phi) * yy
    p = so.Params()
    hist, _ = so.orientation_histogram(L, 30, 30, 2.1, p)
    angles, _ = so.orientation_peaks(hist, p)
    b = phi_deg / 10.0
    j0 = math.floor(b)
    f = b - j0
    if f < 0.5:
        expect = (j0 + 0.5 * f / (1 - f)) * 10.0
    else:
        g = 1.0 - f
        expect = (j0 + 1 - 0.5 * g / (1 - g)) * 10.0
    assert len(angles) == 1
    d = abs(angles[0] - expect % 360.0) % 360.0
    assert min(d, 360 - d) < 1e-9


def test_orientation_peaks_secondary_and_ties():
    p = so.Params()
    h = np.zeros(36)
    h[3], h[20] = 1.0, 0.85
    angles, m = so.orientation_peaks(h, p)
    assert angles == [30.0, 200.0]
    h[20] = 0.7
    assert so.orientation_peaks(h, p)[0] == [30.0]
    # two equal neighbours: no strict maximum, the decision margin is zero
    h = np.zeros(36)
    h[3] = h[4] = 1.0
    angles, m = so.orientation_peaks(h, p)
    assert angles == [] and m == 0.0


# ---------------------------------------------------------------- P10 rotation

def test_rot90_permutes_keypoints_and_keeps_descriptors():
    rng = np.random.default_rng(7)
    h, w = 97, 129
    from paper_2605_17869_amd import synth
    img = synth.blob_image(11, h, w, 80)
    p = p_default(n_octaves=3)
    a = oracle.sift(img, p)
    b = oracle.sift(np.ascontiguousarray(np.rot90(img)), p)
    dec_a = {(e["o"], e["i0"], e["r0"], e["c0"]): e for e in a.log}
    mapped = 0
    for k, kp in enumerate(a.keypoints):
        key = (kp["octave"], kp["src_layer"], kp["src_iy"], kp["src_ix"])
        e = dec_a[key]
        if min(e.get(m, 1) for m in ("m_pre", "m_ext", "m_move", "m_con", "m_edge",
                                     "m_peak", "m_rad")) < 1e-6:
            continue
        x2, y2 = kp["y"], (w - 1) - kp["x"]
        ang2 = (kp["angle"] - 90.0) % 360.0
        hit = [j for j, q in enumerate(b.keypoints)
               if abs(q["x"] - x2) < 1e-7 and abs(q["y"] - y2) < 1e-7
               and min(abs(q["angle"] - ang2) % 360, 360 - abs(q["angle"] - ang2) % 360) < 1e-7]
        assert len(hit) == 1, f"keypoint {k} has no rotated counterpart"
        assert np.max(np.abs(b.descriptors[hit[0]] - a.descriptors[k])) < 1e-9
        mapped += 1
    assert mapped >= max(15, int(0.9 * len(a.keypoints)))
    assert len(a.keypoints) == len(b.keypoints)


def test_rot90_upright_descriptor_is_permuted():
    from paper_2605_17869_amd import synth
    h, w = 97, 129
    img = synth.blob_image(12, h, w, 80)
    p = p_default(n_octaves=3, upright=1)
    a = oracle.sift(img, p)
    b = oracle.sift(np.ascontiguousarray(np.rot90(img)), p)
    perm = np.zeros(128, dtype=int)
    for rho in range(4):
        for kap in range(4):
            for o in range(8):
                perm[((3 - kap) * 4 + rho) * 8 + (o - 2) % 8] = (rho * 4 + kap) * 8 + o
    checked = 0
    for k, kp in enumerate(a.keypoints):
        x2, y2 = kp["y"], (w - 1) - kp["x"]
        hit = [j for j, q in enumerate(b.keypoints)
               if abs(q["x"] - x2) < 1e-7 and abs(q["y"] - y2) < 1e-7]
        if len(hit) != 1:
            continue
        assert np.max(np.abs(b.descriptors[hit[0]] - a.descriptors[k][perm])) < 1e-9
        checked += 1
    assert checked >= max(15, int(0.9 * len(a.keypoints)))


# ---------------------------------------------------------------- P11 / P12 descriptor

def test_descriptor_norms_and_dsp_identity():
    from paper_2605_17869_amd import synth
    img = synth.blob_image(13, 97, 129, 40)
    p = p_default(n_octaves=3)
    r1 = oracle.sift(img, p)
    d = r1.descriptors
    assert len(d) > 10
    assert np.all(d >= 0) and np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-12)
    p2 = p_default(n_octaves=3, dsp_scales=(1.0,))
    assert np.array_equal(oracle.sift(img, p2).descriptors, d)
    p3 = p_default(n_octaves=3, rootsift=1, dsp_scales=(0.5, 1.0, 2.0))
    d3 = oracle.sift(img, p3).descriptors
    assert np.allclose(np.linalg.norm(d3, axis=1), 1.0, atol=1e-12)
    # RootSIFT of the averaged raw histograms, checked step by step on one keypoint
    res = oracle.sift(img, p3, keep_octaves=True)
    kp = res.keypoints[0]
    e = [x for x in res.log if (x["o"], x["i0"], x["r0"], x["c0"]) ==
         (kp["octave"], kp["src_layer"], kp["src_iy"], kp["src_ix"])][0]
    oc = [o for o in res.octaves if o.o == kp["octave"]][0]
    raws = [so.raw_descriptor(oc.L[e["i"]], e["r"], e["c"], e["x_oct"], e["y_oct"],
                              e["sigma_oct"], float(kp["angle"]), s, p3) for s in (0.5, 1.0, 2.0)]
    v = sum(raws) / 3
    v = v / np.linalg.norm(v)
    v = np.minimum(v, 0.2)
    v = v / np.linalg.norm(v)
    v = np.sqrt(v / v.sum())
    assert np.max(np.abs(v - res.descriptors[0])) < 1e-12


def test_raw_descriptor_equals_per_sample_accumulation():
    rng = np.random.default_rng(9)
    L = rng.random((40, 44))
    p = so.Params()
    r, c, x_oct, y_oct, sig, ang = 20, 21, 21.3, 19.8, 1.7, 37.0
    fast = so.raw_descriptor(L, r, c, x_oct, y_oct, sig, ang, 1.0, p)
    slow = np.zeros(128)
    th = math.radians(ang)
    wc = 3.0 * sig
    rad = math.ceil(math.sqrt(2) * 2.5 * wc)
    for rr in range(r - rad, r + rad + 1):
        for cc in range(c - rad, c + rad + 1):
            if not (1 <= rr <= 38 and 1 <= cc <= 42):
                continue
            u, v = cc - x_oct, rr - y_oct
            xr = (math.cos(th) * u + math.sin(th) * v) / wc
            yr = (-math.sin(th) * u + math.cos(th) * v) / wc
            cb, rb = xr + 1.5, yr + 1.5
            if not (-1 < rb < 4 and -1 < cb < 4):
                continue
            gx = L[rr, cc + 1] - L[rr, cc - 1]
            gy = L[rr + 1, cc] - L[rr - 1, cc]
            mag = math.hypot(gx, gy)
            ob = ((math.atan2(gy, gx) - th) % (2 * math.pi)) * 8 / (2 * math.pi)
            wgt = mag * math.exp(-(xr * xr + yr * yr) / 8.0)
            for dr in (0, 1):
                for dc in (0, 1):
                    for do in (0, 1):
                        row, col = math.floor(rb) + dr, math.floor(cb) + dc
                        if not (0 <= row < 4 and 0 <= col < 4):
                            continue
                        ori = (math.floor(ob) + do) % 8
                        fr, fc, fo = rb - math.floor(rb), cb - math.floor(cb), ob - math.floor(ob)
                        wt = (fr if dr else 1 - fr) * (fc if dc else 1 - fc) * (fo if do else 1 - fo)
                        slow[(row * 4 + col) * 8 + ori] += wgt * wt
    assert np.max(np.abs(fast - slow)) < 1e-12


# ---------------------------------------------------------------- ordering / cap

def test_canonical_order_and_cap():
    from paper_2605_17869_amd import synth
    img = synth.blob_image(14, 97, 129, 40)
    p = p_default(n_octaves=3)
    full = oracle.sift(img, p)
    keys = [(int(k["octave"]), int(k["src_layer"]), int(k["src_iy"]), int(k["src_ix"]))
            for k in full.keypoints]
    assert keys == sorted(keys)
    capped = oracle.sift(img, p_default(n_octaves=3, max_keypoints=7))
    assert capped.n_found == len(full.keypoints)
    assert len(capped.keypoints) == 7
    assert np.array_equal(capped.descriptors, full.descriptors[:7])


def test_image_too_small_raises():
    with pytest.raises(ValueError):
        so.scale_space(np.zeros((40, 40), np.float32), p_default(n_octaves=4))


def test_upsample_limit_drops_octave_minus_one_above_the_size():
    """The VRAM-adaptive policy: with upsample on and a pixel limit, an image
    above the limit is extracted exactly as with upsample off, one at or below
    it exactly as with upsample on."""
    from paper_2605_17869_amd import synth
    img = synth.blob_image(15, 97, 129, 40)            # 12513 pixels
    on = oracle.sift(img, p_default(n_octaves=2, upsample=1))
    off = oracle.sift(img, p_default(n_octaves=2, upsample=0))
    assert len(on.keypoints) != len(off.keypoints)
    above = oracle.sift(img, p_default(n_octaves=2, upsample=1, upsample_max_pixels=12512))
    at = oracle.sift(img, p_default(n_octaves=2, upsample=1, upsample_max_pixels=12513))
    assert np.array_equal(above.keypoints, off.keypoints)
    assert np.array_equal(above.descriptors, off.descriptors)
    assert np.array_equal(at.keypoints, on.keypoints)
    assert min(above.keypoints["octave"]) == 0 and min(at.keypoints["octave"]) == -1


# ---------------------------------------------------------------------------
# fp16 pyramid storage (section 3.2, "GPU Pipeline Stages")

def _fp16_pair(img, **kw):
    from paper_2605_17869_amd import synth  # noqa: F401  (inputs only)
    p32 = so.Params(n_octaves=3, **kw)
    p16 = so.Params(n_octaves=3, pyramid_fp16=1, **kw)
    return so.scale_space(img, p32), so.scale_space(img, p16)


@pytest.mark.parametrize("up", [0, 1])
def test_fp16_storage_keeps_the_first_octave_and_rounds_the_rest(up):
    from paper_2605_17869_amd import synth
    img = synth.blob_image(77, 90, 120, 40)
    o32, o16 = _fp16_pair(img, upsample=up)
    # the first octave is untouched, bit for bit
    np.testing.assert_array_equal(o32[0].L, o16[0].L)
    for a, b in zip(o32[1:], o16[1:]):
        centred = b.L - 0.5
        # every stored value is an fp16 number
        np.testing.assert_array_equal(centred, centred.astype(np.float16).astype(np.float64))
        # each of the s+3 levels adds at most half an fp16 ulp of |L - 1/2| <= 1/2
        # (2^-12 for values in [1/4, 1/2)), and a unit-sum non-negative blur
        # never grows an error: levels stay within (octave count x (s+3)) half-ulps
        bound = (a.o - o32[0].o) * len(a.L) * 2.0 ** -12
        assert np.max(np.abs(a.L - b.L)) <= bound
        assert np.max(np.abs(a.L - b.L)) > 0.0


def test_fp16_storage_of_a_constant_image_is_exact():
    # blurring a constant leaves it constant up to the fp64 tap sum; stored in
    # fp16 the later octaves hold exactly mid-grey
    img = np.full((60, 80), 0.5, np.float32)
    o32, o16 = _fp16_pair(img)
    for a, b in zip(o32, o16):
        assert np.max(np.abs(a.L - b.L)) < 1e-15
    for b in o16[1:]:
        assert np.all(b.L == 0.5)
    assert len(so.sift(img, so.Params(n_octaves=3, pyramid_fp16=1)).keypoints) == 0


def test_fp16_storage_leaves_first_octave_keypoints_unchanged():
    from paper_2605_17869_amd import synth
    img = synth.blob_image(78, 160, 200, 90)
    r32 = so.sift(img, so.Params(n_octaves=3))
    r16 = so.sift(img, so.Params(n_octaves=3, pyramid_fp16=1))

    def first(r):
        k = r.keypoints
        sel = k["octave"] == 0
        return k[sel].tobytes(), r.descriptors[sel].tobytes(), int(sel.sum())

    assert first(r32) == first(r16) and first(r32)[2] > 5

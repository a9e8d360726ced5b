"""Pins of the oracle's decision margins, window weights and descriptor
normalisation (CPU only).

Every accept/reject decision of the oracle carries a relative margin, and the
parity checker exempts a candidate whose margin is at most 1e-4.  A margin
computed too large would hide a real mismatch; one computed too small would
silently widen the exemption.  Each margin is therefore pinned here on crafted
inputs that put the decision a known relative distance eps from its threshold:
the margin must equal the value derived by hand for that construction, and the
decision must flip exactly where the margin goes through zero.

The orientation window and descriptor weights are pinned with single-spike
levels: a level that is zero except for one pixel has exactly four non-zero
central-difference gradients, of unit magnitude and at 0, 90, 180 and 270
degrees, so every histogram entry they produce is one Gaussian weight whose
value is known in closed form.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import sift_oracle as so

EPS = (-3e-2, -1e-3, -1e-5, 1e-5, 1e-3, 3e-2)


def params(**kw):
    p = so.Params()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def quadratic_octave(centre, hess, peak, shape=(5, 31, 33)):
    """DoG stack sampled from q(p) = peak + 1/2 (p - centre)^T H (p - centre)
    with p = (x, y, s) = (column, row, layer): central differences are exact on
    a quadratic, so the refinement's step, extremum value and Hessian are all
    known in closed form."""
    s_, h, w = shape
    ii, rr, cc = np.meshgrid(np.arange(s_), np.arange(h), np.arange(w), indexing="ij")
    d = np.stack([cc - centre[0], rr - centre[1], ii - centre[2]], axis=-1).astype(np.float64)
    q = peak + 0.5 * np.einsum("...a,ab,...b->...", d, np.asarray(hess, dtype=np.float64), d)
    L = np.zeros((s_ + 1, h, w))
    L[1:] = np.cumsum(q, axis=0)
    return so.Octave(0, L, q)


# ---------------------------------------------------------------- candidates

@pytest.mark.parametrize("eps", EPS)
def test_pregate_margin_is_the_relative_distance_to_the_gate(eps):
    p = params(border=2)
    gate = p.prefilter_ratio * p.contrast_threshold
    D = np.zeros((3, 9, 9))
    for sign in (1.0, -1.0):
        D[1, 4, 4] = sign * gate * (1.0 + eps)
        m = so.pixel_margins(D, 1, 4, 4, p)
        assert m["m_pre"] == pytest.approx(abs(eps), rel=1e-6, abs=1e-12)
        # an isolated peak: only the pre-gate decides
        assert bool(so.candidate_mask(D, 1, p)[4, 4]) == (eps > 0)


NEIGHBOURS = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
              if (a, b, c) != (0, 0, 0)]


@pytest.mark.parametrize("near", NEIGHBOURS)
def test_extremum_margin_names_the_closest_neighbour(near):
    """Centre v = 0.05, every neighbour 0.02 below it except `near`, which is
    delta below (an extremum, margin delta / v) or delta above (not one; the
    value must rise by delta to become the maximum, margin delta / v)."""
    p = params(border=2)
    v = 0.05
    for delta, is_ext in ((0.004, True), (0.0001, True), (0.004, False), (0.0001, False)):
        D = np.full((3, 9, 9), -1.0)
        D[:, 3:6, 3:6] = v - 0.02
        D[1, 4, 4] = v
        D[1 + near[0], 4 + near[1], 4 + near[2]] = v - delta if is_ext else v + delta
        m = so.pixel_margins(D, 1, 4, 4, p)
        assert m["m_ext"] == pytest.approx(delta / v, rel=1e-9)
        assert bool(so.candidate_mask(D, 1, p)[4, 4]) == is_ext
        # the mirror image (a minimum) has the same margin
        m2 = so.pixel_margins(-D, 1, 4, 4, p)
        assert m2["m_ext"] == pytest.approx(delta / v, rel=1e-9)
        assert bool(so.candidate_mask(-D, 1, p)[4, 4]) == is_ext


# ---------------------------------------------------------------- refinement

H0 = np.array([[0.02, 0.003, 0.001], [0.003, 0.03, 0.002], [0.001, 0.002, 0.05]])
START = (15, 13, 2)          # column, row, layer of the candidate


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("eps", [-0.02, -1e-3, 1e-3, 0.02])
def test_step_margin_at_half_a_pixel(axis, eps):
    """Extremum 0.5 + eps from the start along one axis (the others exactly on
    the start): the first solve gives |x^| = 0.5 + eps there.  eps > 0 moves
    one step, after which |x^| = 0.5 - eps; eps < 0 stops at once.  Either way
    the closest approach to a rounding boundary is |eps|, relative to 0.5."""
    H = np.diag(np.diag(H0))
    centre = [float(v) for v in START]
    centre[axis] += 0.5 + eps
    oc = quadratic_octave(centre, H, peak=-0.05)
    res = so.refine(oc, START[2], START[1], START[0], params(border=3))
    assert res["status"] == "ok"
    assert res["m_move"] == pytest.approx(abs(eps) / 0.5, rel=1e-6)
    moved = [0, 0, 0]
    moved[axis] = 1 if eps > 0 else 0
    assert (res["c"], res["r"], res["i"]) == (START[0] + moved[0], START[1] + moved[1],
                                              START[2] + moved[2])


def test_step_margin_is_relative_to_the_boundary_crossed():
    """x^ = 1.5 + eps rounds to 2; the margin of that decision is eps / 1.5,
    and the next solve (x^ = -0.5 + eps) has eps / 0.5: the minimum is eps / 1.5."""
    eps = 0.01
    H = np.diag([0.02, 0.03, 0.05])
    oc = quadratic_octave((START[0] + 1.5 + eps, START[1], START[2]), H, peak=-0.05)
    res = so.refine(oc, START[2], START[1], START[0], params(border=3))
    assert res["status"] == "ok" and res["c"] == START[0] + 2
    assert res["m_move"] == pytest.approx(eps / 1.5, rel=1e-6)


@pytest.mark.parametrize("eps", EPS)
def test_contrast_margin(eps):
    """The extremum value of the quadratic is `peak` exactly, whatever the
    sub-pixel offset (D + 1/2 g.x^ at the solution); peak = -T (1 + eps)."""
    p = params(border=3)
    T = p.contrast_threshold
    centre = (START[0] + 0.2, START[1] - 0.3, START[2] + 0.1)
    oc = quadratic_octave(centre, H0, peak=-T * (1.0 + eps))
    res = so.refine(oc, START[2], START[1], START[0], p)
    assert res["contrast"] == pytest.approx(-T * (1.0 + eps), rel=1e-12)
    assert res["m_con"] == pytest.approx(abs(eps), rel=1e-6, abs=1e-12)
    assert (res["status"] == "ok") == (eps > 0)
    if eps < 0:
        assert res["status"] == "contrast"


def rotated_hessian(a, rho, angle, hs=0.05):
    """Spatial Hessian with eigenvalues a and a * rho, eigenvectors rotated by
    `angle` (trace and determinant do not depend on it), scale curvature hs."""
    c, s = math.cos(angle), math.sin(angle)
    R = np.array([[c, -s], [s, c]])
    H2 = R @ np.diag([a, a * rho]) @ R.T
    H = np.zeros((3, 3))
    H[:2, :2] = H2
    H[2, 2] = hs
    return H


@pytest.mark.parametrize("r_e", [10.0, 5.0])
@pytest.mark.parametrize("eps", [-0.02, -1e-3, 1e-3, 0.02])
@pytest.mark.parametrize("angle", [0.0, 0.6])
def test_edge_margin_near_the_curvature_ratio_bound(r_e, eps, angle):
    """Curvature ratio rho = r (1 + eps).  The edge inequality r tr^2 <
    (r+1)^2 det has relative slack N(rho) / ((r+1)^2 rho) with N(rho) =
    (r+1)^2 rho - r (1+rho)^2, whose derivative at rho = r is (r+1)(1-r);
    to first order the margin is (r-1)/(r+1) |eps|.  A rotated Hessian (a
    non-zero mixed derivative) gives the same margin."""
    p = params(border=3, edge_ratio=r_e)
    a = 0.01
    H = rotated_hessian(a, r_e * (1.0 + eps), angle)
    oc = quadratic_octave((START[0], START[1], START[2]), H, peak=-0.05)
    res = so.refine(oc, START[2], START[1], START[0], p)
    # in terms of the eigenvalues (the oracle works from finite differences
    # of the rotated quadratic): tr = a (1 + rho), det = a^2 rho
    rho = r_e * (1.0 + eps)
    exact = abs((r_e + 1.0) ** 2 * rho - r_e * (1.0 + rho) ** 2) / ((r_e + 1.0) ** 2 * rho)
    assert res["m_edge"] == pytest.approx(exact, rel=1e-6)
    first_order = (r_e - 1.0) / (r_e + 1.0) * abs(eps)
    assert res["m_edge"] == pytest.approx(first_order, rel=3 * abs(eps) + 1e-6)
    assert (res["status"] == "ok") == (eps < 0)


def test_edge_margin_of_a_saddle():
    """det < 0 (a saddle): rejected; margin |det| / (|Dxx Dyy| + Dxy^2),
    which is 1 for a diagonal Hessian."""
    H = np.diag([0.02, -0.01, 0.05])
    oc = quadratic_octave((START[0], START[1], START[2]), H, peak=-0.05)
    res = so.refine(oc, START[2], START[1], START[0], params(border=3))
    assert res["status"] == "edge" and res["m_edge"] == pytest.approx(1.0)


# ---------------------------------------------------------------- orientation

@pytest.mark.parametrize("eps", [-0.02, -1e-3, 1e-3, 0.02])
def test_secondary_peak_margin(eps):
    """Raw spikes of 1 and x = 0.8 (1 + eps) in isolated bins: after the
    [1/4, 1/2, 1/4] pass they stay peaks of heights 1/2 and x/2, so the second
    is kept iff x >= 0.8, and its ratio margin is (x - 0.8) relative to 1."""
    p = so.Params()
    h = np.zeros(36)
    h[3], h[20] = 1.0, 0.8 * (1.0 + eps)
    angles, m = so.orientation_peaks(h, p)
    assert m == pytest.approx(0.8 * abs(eps), rel=1e-9)
    assert angles == ([30.0, 200.0] if eps > 0 else [30.0])


@pytest.mark.parametrize("delta", [1e-4, 1e-2, 0.2])
def test_local_maximum_margin_after_smoothing(delta):
    """Adjacent raw bins 1 and 1 - delta: the smoothed heights are
    3/4 - delta/4 and 3/4 - delta/2, a gap of delta/4, relative to the
    maximum 3/4 - delta/4; only the first bin is a peak."""
    p = so.Params()
    h = np.zeros(36)
    h[5], h[6] = 1.0, 1.0 - delta
    angles, m = so.orientation_peaks(h, p)
    assert m == pytest.approx(0.25 * delta / (0.75 - 0.25 * delta), rel=1e-9)
    assert len(angles) == 1 and 50.0 <= angles[0] < 60.0


@pytest.mark.parametrize("dq", [-1e-3, -1e-5, 1e-5, 1e-3])
def test_window_radius_margin(dq):
    """q = 3 sigma_w + 1/2 just above or below the integer 10: the radius is
    floor(q) and the margin |q - 10| / q."""
    p = so.Params()
    q = 10.0 + dq
    sigma_oct = (q - 0.5) / (p.ori_radius_factor * p.ori_sigma_factor)
    L = np.zeros((41, 41))
    _, m_rad = so.orientation_histogram(L, 20, 20, sigma_oct, p)
    assert m_rad == pytest.approx(abs(dq) / q, rel=1e-6)


def spike(shape, y, x):
    L = np.zeros(shape)
    L[y, x] = 1.0
    return L


def spike_samples(y, x):
    """The four pixels with a non-zero central difference around a unit spike
    at (y, x), with their gradient angles in degrees (y points down)."""
    return [((y, x - 1), 0.0), ((y, x + 1), 180.0), ((y - 1, x), 90.0), ((y + 1, x), 270.0)]


@pytest.mark.parametrize("sigma_oct", [2.1, 1.7])
def test_orientation_window_weights_from_a_spike(sigma_oct):
    """Raw orientation histogram of a single spike placed at many offsets from
    the keypoint: each of its four unit gradients lands on a bin centre
    (0, 9, 18, 27) with the Gaussian weight exp(-d^2 / (2 (1.5 sigma)^2)) of
    its offset d, and only if the offset lies in the square of radius
    floor(4.5 sigma + 1/2)."""
    p = so.Params()
    sw = 1.5 * sigma_oct
    R = math.floor(3.0 * sw + 0.5)
    r0 = c0 = 30
    for (dy, dx) in [(0, 0), (2, -3), (-5, 4), (R, 0), (R + 1, 0), (0, R), (-R, R - 1), (7, -8)]:
        y, x = r0 + dy, c0 + dx
        L = spike((61, 61), y, x)
        hist, _ = so.orientation_histogram(L, r0, c0, sigma_oct, p)
        expect = np.zeros(36)
        for (py, px), ang in spike_samples(y, x):
            oy, ox = py - r0, px - c0
            if max(abs(oy), abs(ox)) <= R:
                expect[int(round(ang / 10.0)) % 36] += math.exp(-(oy * oy + ox * ox) / (2 * sw * sw))
        assert np.max(np.abs(hist - expect)) < 1e-12, (dy, dx)


# ---------------------------------------------------------------- descriptor

@pytest.mark.parametrize("angle", [0.0, 90.0])
@pytest.mark.parametrize("sy,sx", [(30, 30), (31, 31), (30, 31), (29, 32), (32, 29), (31, 30)])
def test_descriptor_weights_from_a_spike(angle, sy, sx):
    """Cell width 3 sigma = 1 px (sigma = 1/3) and the sub-pixel centre at
    (30.5, 30.5): every pixel of the 4 x 4 block 29..32 is a cell centre, so
    each gradient sample falls in exactly one cell and, its angle being a
    multiple of 90 degrees, in exactly one orientation bin.  The entry it
    makes is exp(-(xr^2 + yr^2) / 8): the Gaussian of sigma = 2 cells (half
    the grid width) at its rotated cell coordinates."""
    p = so.Params()
    L = spike((61, 61), sy, sx)
    raw = so.raw_descriptor(L, 30, 30, 30.5, 30.5, 1.0 / 3.0, angle, 1.0, p)
    th = math.radians(angle)
    expect = np.zeros(128)
    for (py, px), ga in spike_samples(sy, sx):
        u, v = px - 30.5, py - 30.5
        xr = math.cos(th) * u + math.sin(th) * v
        yr = -math.sin(th) * u + math.cos(th) * v
        col, row = round(xr + 1.5), round(yr + 1.5)
        if not (0 <= row < 4 and 0 <= col < 4):
            continue
        ori = int(round(((ga - angle) % 360.0) / 45.0)) % 8
        expect[(row * 4 + col) * 8 + ori] += math.exp(-(xr * xr + yr * yr) / 8.0)
    assert np.count_nonzero(expect) >= 2
    assert np.max(np.abs(raw - expect)) < 1e-12


def test_descriptor_angle_90_uses_the_rotated_grid():
    """With the keypoint at 90 degrees the grid's x axis points down the image:
    a spike right of the centre lies in the top row of cells, and a gradient
    pointing down (90 degrees) is orientation bin 0."""
    p = so.Params()
    L = spike((61, 61), 30, 31)          # gradients at (30,30):0, (30,32):180, (29,31):90, (31,31):270
    raw = so.raw_descriptor(L, 30, 30, 30.5, 30.5, 1.0 / 3.0, 90.0, 1.0, p)
    # sample (31, 31), angle 270: u = 0.5, v = 0.5 -> xr = 0.5, yr = -0.5: row 1, col 2, bin 4
    assert raw[(1 * 4 + 2) * 8 + 4] == pytest.approx(math.exp(-0.5 / 8.0), rel=1e-12)
    # sample (29, 31), angle 90: u = 0.5, v = -1.5 -> xr = -1.5, yr = -0.5: row 1, col 0, bin 0
    assert raw[(1 * 4 + 0) * 8 + 0] == pytest.approx(math.exp(-2.5 / 8.0), rel=1e-12)


def test_descriptor_domain_size_scales_the_cell():
    """Domain size 2 doubles the cell (2 px): with the centre on the integer
    pixel (30, 30) the cell centres are the odd offsets +-1, +-3, and a sample
    there again fills one cell, now with exp(-(offset / 2)^2 / 8) per axis."""
    p = so.Params()
    L = spike((61, 61), 31, 32)          # sample (31, 31) angle 0: offsets u = 1, v = 1
    raw = so.raw_descriptor(L, 30, 30, 30.0, 30.0, 1.0 / 3.0, 0.0, 2.0, p)
    # xr = yr = 0.5 cells: row 2, col 2, bin 0
    assert raw[(2 * 4 + 2) * 8 + 0] == pytest.approx(math.exp(-0.5 / 8.0), rel=1e-12)
    # sample (31, 33), angle 180: u = 3, v = 1 -> xr = 1.5, yr = 0.5: row 2, col 3, bin 4
    assert raw[(2 * 4 + 3) * 8 + 4] == pytest.approx(math.exp(-2.5 / 8.0), rel=1e-12)


def test_normalise_clamp_properties():
    """L2 -> clamp -> L2: components that the clamp does not touch keep their
    ratios, the clamped ones end equal and largest, and the result has unit
    norm; with every component under the clamp the result is h / |h|."""
    p = so.Params()
    rng = np.random.default_rng(3)
    h = rng.random(128) * 0.1
    h[[5, 77]] = [10.0, 6.0]
    v = so.normalise(h, p)
    assert np.linalg.norm(v) == pytest.approx(1.0, abs=1e-14)
    clamped = h / np.linalg.norm(h) > p.desc_clamp
    assert set(np.nonzero(clamped)[0]) == {5, 77}
    assert v[5] == v[77] == v.max()
    free = ~clamped
    ratio = v[free] / h[free]
    assert np.max(ratio) - np.min(ratio) < 1e-12 * np.max(ratio)
    # worked example: one entry of 10 and 99 of 1 (v0 = 10 / sqrt(199) > 0.2)
    h2 = np.zeros(128)
    h2[0], h2[1:100] = 10.0, 1.0
    v2 = so.normalise(h2, p)
    n2 = math.sqrt(0.04 + 99.0 / 199.0)
    assert v2[0] == pytest.approx(0.2 / n2, rel=1e-12)
    assert v2[1] == pytest.approx((1.0 / math.sqrt(199.0)) / n2, rel=1e-12)
    # nothing above the clamp: plain L2 normalisation
    h3 = np.ones(128)
    assert np.allclose(so.normalise(h3, p), h3 / math.sqrt(128.0), rtol=0, atol=1e-15)
    # RootSIFT: squares are the clamped descriptor over its L1 norm
    pr = params(rootsift=1)
    r = so.normalise(h, pr)
    assert np.allclose(r * r, v / v.sum(), rtol=0, atol=1e-15)
    assert np.linalg.norm(r) == pytest.approx(1.0, abs=1e-14)
    assert np.array_equal(so.normalise(np.zeros(128), p), np.zeros(128))


# ---------------------------------------------------------------- caps

def test_candidate_cap_refines_the_canonical_prefix():
    from paper_2605_17869_amd import synth
    img = synth.blob_image(14, 97, 129, 60)
    full = oracle.sift(img, params(n_octaves=3))
    cut = oracle.sift(img, params(n_octaves=3, max_candidates=9))
    assert full.n_candidates == cut.n_candidates == len(full.log) > 9
    assert len(cut.log) == 9
    keys = lambda log: [(e["o"], e["i0"], e["r0"], e["c0"]) for e in log]
    assert keys(cut.log) == keys(full.log)[:9]
    n = len(cut.keypoints)
    assert np.array_equal(cut.descriptors, full.descriptors[:n])

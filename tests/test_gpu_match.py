"""Matching on the matrix cores (sift_match_batch through the C ABI) against
the FP64 reference matcher, plus determinism, batch invariance, device-side
counts and an end-to-end check on warped image pairs.  Needs an MI355X."""
import numpy as np
import pytest

from oracle import match_oracle as mo
from paper_2605_17869_amd import synth
from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


def gpu_match(pairs_np, ratio=0.8, counts=None):
    torch = require_gpu()
    from paper_2605_17869_amd import match_batch
    args = []
    for k, (a, b) in enumerate(pairs_np):
        ta = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32).reshape(-1, 128)).cuda()
        tb = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float32).reshape(-1, 128)).cuda()
        ca = cb = None
        if counts is not None and counts[k] is not None:
            ca = torch.tensor([counts[k][0]], dtype=torch.int32, device="cuda")
            cb = torch.tensor([counts[k][1]], dtype=torch.int32, device="cuda")
        args.append((ta, ca, tb, cb))
    outs = match_batch(args, ratio=ratio)
    torch.cuda.synchronize()
    return [m.host() for m in outs]


def check_against_oracle(a, b, rec, n_found, ratio=0.8):
    """Decisive rows: same keep decision and partner, similarity within the
    accumulation bound, squared distance within 4x it.  Every GPU match is an
    oracle match or sits on a marginal row.  Order: ascending query."""
    ref = mo.match(a, b, ratio)
    q = rec["query"].astype(np.int64)
    assert np.all(np.diff(q) > 0), "matches must come in ascending query order"
    assert n_found == len(rec)
    gpu = {int(i): k for k, i in enumerate(q)}
    ref_rows = {int(i): k for k, i in enumerate(ref.pairs[:, 0])}
    marginal = 0
    for i in range(len(a)):
        if not ref.decisive[i]:
            marginal += 1
            continue
        assert (i in gpu) == (i in ref_rows), f"row {i}: keep decision differs"
        if i in gpu:
            k, kr = gpu[i], ref_rows[i]
            assert int(rec["train"][k]) == int(ref.pairs[kr, 1])
            assert abs(float(rec["similarity"][k]) - ref.sim[kr]) <= mo.TOL
            d2_gpu = float(rec["distance"][k]) ** 2
            assert abs(d2_gpu - ref.dist[kr] ** 2) <= 4 * mo.TOL + 1e-6
    for i in gpu:
        if i not in ref_rows:
            assert not ref.decisive[i], f"row {i}: GPU kept a pair the oracle decisively rejects"
    return len(ref.pairs), marginal


@pytest.mark.parametrize("seed,na,nb,nc,noise", [
    (101, 300, 400, 200, 0.05),      # clean copies: every common row matched
    (102, 1000, 700, 500, 0.12),     # noisy: many rejections, ragged tails
    (103, 129, 257, 100, 0.12),      # one row past a 128-row tile
    (104, 1, 5, 1, 0.1),             # single query row
    (105, 5, 1, 1, 0.1),             # single candidate: D2 = 4
    (106, 2000, 2000, 1500, 0.1),    # c3-sized sets
])
def test_matches_equal_oracle(seed, na, nb, nc, noise):
    a, b, _ = synth.descriptor_sets(seed, na, nb, nc, noise)
    (rec, nf), = gpu_match([(a, b)])
    n_ref, marginal = check_against_oracle(a, b, rec, nf)
    say(f"seed {seed}: {na}x{nb}: gpu {len(rec)} oracle {n_ref} marginal rows {marginal}")
    assert len(rec) > 0


def test_ratio_parameter_and_boundary():
    a = np.zeros((1, 128), np.float32)
    a[0, 0] = 1.0
    for x1, keep in [(0.6796875, False), (0.68017578125, True)]:
        b = np.zeros((2, 128), np.float32)
        b[0, 0], b[1, 0] = x1, 0.5
        (rec, nf), = gpu_match([(a, b)], ratio=0.8)
        assert (len(rec) == 1) == keep
    a2, b2, _ = synth.descriptor_sets(107, 400, 400, 300, 0.12)
    for r in (0.6, 0.9, 1.0):
        (rec, nf), = gpu_match([(a2, b2)], ratio=r)
        check_against_oracle(a2, b2, rec, nf, ratio=r)


def test_batch_equals_single_and_is_deterministic():
    sets = [synth.descriptor_sets(200 + k, 150 + 97 * k, 300 - 41 * k, 100, 0.12)[:2]
            for k in range(5)]
    batch = gpu_match(sets)
    for k, (a, b) in enumerate(sets):
        (rec, nf), = gpu_match([(a, b)])
        assert rec.tobytes() == batch[k][0].tobytes() and nf == batch[k][1]
    again = gpu_match(sets)
    for x, y in zip(batch, again):
        assert x[0].tobytes() == y[0].tobytes()


def test_device_counts_limit_the_rows():
    a, b, _ = synth.descriptor_sets(300, 700, 600, 400, 0.12)
    (rec, nf), = gpu_match([(a, b)], counts=[(450, 333)])
    check_against_oracle(a[:450], b[:333], rec, nf)
    (rec0, nf0), = gpu_match([(a, b)], counts=[(0, 333)])
    assert len(rec0) == 0 and nf0 == 0


def test_warped_pairs_end_to_end():
    """Extraction and matching chained on the device (keypoint counts passed
    as device pointers) for a 1600x1066 image and its seeded affine copy:
    matched keypoints land where the known map sends them.  A property of the
    output, not parity: the matcher's parity cases use seeded descriptor sets."""
    torch = require_gpu()
    from paper_2605_17869_amd import Extractor, match
    wl = synth.workload(3, n_images=2)
    img = wl.image(0)
    warped, fwd = synth.warped_copy(img, synth.workload_seed(3, 0, True))
    ex = Extractor(wl.settings)
    fa = ex.extract(torch.from_numpy(img).cuda())
    fb = ex.extract(torch.from_numpy(warped).cuda())
    m = match(fa.descriptors, fb.descriptors, count_a=fa.counters[0:1], count_b=fb.counters[0:1])
    torch.cuda.synchronize()
    rec, nf = m.host()
    ka = fa.host()[0]
    kb = fb.host()[0]
    pa = np.stack([ka["x"], ka["y"], np.ones(len(ka))], 1)[rec["query"]]
    pb = np.stack([kb["x"], kb["y"]], 1)[rec["train"]]
    err = np.linalg.norm(pa @ fwd.T - pb, axis=1)
    inl = float(np.mean(err < 3.0))
    say(f"{len(ka)} / {len(kb)} keypoints, {len(rec)} matches, inlier fraction {inl:.3f}")
    assert len(rec) > 100 and inl > 0.8
    assert np.all(np.diff(rec["query"]) > 0)

"""Pins of the reference matcher (oracle/match_oracle.py) against what the
matching step's definition fixes (Section 3.4, "Descriptor Matching", backend
(1): fp16 similarity, ratio test, mutual consistency): closed-form similarities
of fp16-exact vectors, the ratio boundary r^2 on both sides, mutual and tie
cases built by hand, brute-force loops on tiny sets, and the symmetry of the
test under swapping the two sets.  CPU only."""
import numpy as np
import pytest

from oracle import match_oracle as mo
from paper_2605_17869_amd import synth


def e(k, dim=128, scale=1.0):
    v = np.zeros(dim, dtype=np.float32)
    v[k] = scale
    return v


@pytest.mark.parametrize("seed,na,nb,nc,noise", [
    (1, 12, 15, 8, 0.5), (2, 9, 9, 9, 0.8), (3, 15, 6, 4, 0.3), (4, 7, 11, 0, 0.1),
    (5, 14, 14, 10, 1.5)])
def test_vectorised_equals_bruteforce(seed, na, nb, nc, noise):
    a, b, _ = synth.descriptor_sets(seed, na, nb, nc, noise)
    got = [tuple(p) for p in mo.match(a, b).pairs.tolist()]
    assert got == mo.match_bruteforce(a, b)


def test_similarity_is_exact_fp16_dot_product():
    # components exactly representable in fp16: the similarity is their exact
    # dot product, and fp32 inputs are rounded to nearest-even fp16 first
    a = np.zeros((1, 128), np.float32)
    b = np.zeros((2, 128), np.float32)
    a[0, :3] = [0.5, 0.25, 0.125]
    b[0, :3] = [0.75, 0.5, 1.0]
    b[1, 0] = 1.0 + 2.0 ** -12          # rounds to 1.0 in fp16 (ties to even)
    s = mo.similarity(a, b)
    assert s[0, 0] == 0.5 * 0.75 + 0.25 * 0.5 + 0.125 * 1.0
    assert s[0, 1] == 0.5
    assert mo.round_fp16(np.float32([1.0 + 3 * 2.0 ** -12]))[0] == 1.0 + 2.0 ** -10


def test_identical_sets_match_their_permutation():
    a, _, _ = synth.descriptor_sets(11, 40, 1, 0)
    perm = np.random.default_rng(3).permutation(40)
    b = a[perm]
    r = mo.match(a, b)
    inv = np.argsort(perm)
    assert r.pairs.tolist() == [[i, int(inv[i])] for i in range(40)]
    a16 = mo.round_fp16(a)
    np.testing.assert_array_equal(r.sim, np.sum(a16 * a16, axis=1))
    assert np.all(r.decisive)


@pytest.mark.parametrize("x1,keep", [(0.6796875, False), (0.68017578125, True)])
def test_ratio_boundary(x1, keep):
    # a = {e0}; b = {x1 e0, 0.5 e0}: D1 = 2 - 2 x1, D2 = 2 - 2 * 0.5 = 1, and the
    # row test passes iff D1 < r^2 D2 = 0.64 (r = 0.8): the boundary sits at
    # x1 = 0.68, between these two fp16 values.  b's rows see one candidate
    # (D2 = 4), so the column tests pass.
    a = e(0)[None]
    b = np.stack([e(0, scale=x1), e(0, scale=0.5)])
    r = mo.match(a, b, ratio=0.8)
    assert (r.pairs.tolist() == [[0, 0]]) == keep
    # the same two values decide the other way round with the sets swapped
    r2 = mo.match(b, a, ratio=0.8)
    assert (r2.pairs.tolist() == [[0, 0]]) == keep


def test_ratio_squared_in_fp32():
    assert mo.ratio_sq(0.8) == np.float32(float(np.float32(0.8)) ** 2)
    assert mo.ratio_sq(1.0) == np.float32(1.0)


def test_single_candidate_uses_distance_four():
    # one row each way: D2 = 4, so the pair is kept iff D1 < 4 r^2 = 2.56
    a = e(0)[None]
    for x, keep in [(0.0, True), (-0.25, True), (-0.28125, False)]:
        b = e(0, scale=x)[None]
        r = mo.match(a, b, ratio=0.8)
        assert (len(r.pairs) == 1) == keep, x


def test_mutual_check():
    # a0 . b0 = 0.75 is a0's best, but b0 prefers a1 (0.875): no pair for a0;
    # a1 <-> b0 is mutual and passes the ratio tests
    a = np.stack([e(0), e(1)])
    b = np.stack([e(0, scale=0.75) + e(1, scale=0.875), e(2, scale=0.25)])
    r = mo.match(a, b, ratio=0.95)
    assert r.pairs.tolist() == [[1, 0]]
    assert r.log[0]["mutual"] is False


def test_equal_best_similarities_fail_the_ratio_test():
    a = e(0)[None]
    b = np.stack([e(0, scale=0.875), e(0, scale=0.875), e(1)])
    r = mo.match(a, b, ratio=1.0)
    assert r.row_best[0] == 0          # smallest index among equals
    assert len(r.pairs) == 0           # D1 = D2 is not < r^2 D2
    assert r.log[0]["row_gap"] == 0.0


@pytest.mark.parametrize("seed", [7, 8, 9])
def test_swapping_sets_transposes_matches(seed):
    a, b, _ = synth.descriptor_sets(seed, 60, 45, 30, 0.6)
    ab = {tuple(p) for p in mo.match(a, b).pairs.tolist()}
    ba = {(j, i) for i, j in mo.match(b, a).pairs.tolist()}
    assert ab == ba


def test_empty_sets():
    a, b, _ = synth.descriptor_sets(5, 3, 4, 2)
    assert len(mo.match(a[:0], b).pairs) == 0
    assert len(mo.match(a, b[:0]).pairs) == 0


def test_noisy_copies_are_recovered():
    a, b, truth = synth.descriptor_sets(21, 500, 600, 300, 0.05)
    r = mo.match(a, b)
    got = {tuple(p) for p in r.pairs.tolist()}
    assert got == {tuple(t) for t in truth.tolist()}
    assert np.all(np.diff(r.pairs[:, 0]) > 0)

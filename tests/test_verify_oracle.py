"""Pins of the reference verifier (oracle/verify_oracle.py): the closed-form
marginal weight against numerical integration of its definition, the
minimal DLT against a known homography, recovery of the true model and inlier
set from noise-free correspondences with outliers, the effect of the
refinement, degenerate samples, normalisation, and invariance to the order of
the correspondences.  CPU only."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import verify_oracle as vo
from paper_2605_17869_amd import synth


@pytest.mark.parametrize("sigma_max", [1.0, 2.0, 3.5])
def test_marginal_weight_equals_its_integral(sigma_max):
    def integrand(s, r):
        if r > vo.TAU * s:          # truncated at the 0.99 quantile tau * s
            return 0.0
        return r / s ** 2 * math.exp(-r * r / (2.0 * s * s))

    for r in [0.01, 0.3, 1.0, 2.5, vo.TAU * sigma_max * 0.999, vo.TAU * sigma_max * 1.001]:
        num = quad(integrand, 1e-9, sigma_max, args=(r,), points=[r / vo.TAU], limit=200)[0]
        assert abs(float(vo.marginal_weight(r, sigma_max)) - num / sigma_max) < 1e-9, r
    assert float(vo.marginal_weight(np.inf, sigma_max)) == 0.0


def test_tau_is_the_rayleigh_099_quantile():
    assert abs((1.0 - math.exp(-vo.TAU ** 2 / 2.0)) - 0.99) < 1e-15


def test_minimal_dlt_reproduces_a_homography():
    a, b, H, _ = synth.homography_pairs(3, 4, outlier_frac=0.0, noise=0.0)
    Ta, Tb = vo.normaliser(a), vo.normaliser(b)
    an = (np.c_[a, np.ones(4)] @ Ta.T)[:, :2]
    bn = (np.c_[b, np.ones(4)] @ Tb.T)[:, :2]
    A, rhs = vo.dlt_rows(an, bn)
    h = vo.solve8(A, rhs)
    np.testing.assert_allclose(np.linalg.solve(A, rhs), h, rtol=1e-10, atol=1e-12)
    Hest = vo.denormalise(vo.h_matrix(h), Ta, Tb)
    np.testing.assert_allclose(Hest, H, rtol=1e-8, atol=1e-10)


def test_normaliser_centres_and_scales():
    a, *_ = synth.homography_pairs(4, 50)
    T = vo.normaliser(a)
    an = (np.c_[a, np.ones(50)] @ T.T)[:, :2]
    assert np.allclose(an.mean(axis=0), 0.0, atol=1e-12)
    assert abs(np.mean(np.linalg.norm(an, axis=1)) - math.sqrt(2.0)) < 1e-12


def test_exact_inliers_give_the_true_model_and_inlier_set():
    a, b, H, inl = synth.homography_pairs(5, 300, outlier_frac=0.4, noise=0.0)
    res = vo.verify(a, b, synth.sample_numbers(6, 300), sigma_max=2.0)
    np.testing.assert_allclose(res.H, H, rtol=1e-7, atol=1e-9)
    w = vo.marginal_weight(vo.residuals(res.H, a, b), 2.0)
    assert np.array_equal(w > 0, inl | (w > 0))      # every inlier is counted
    assert res.n_inliers >= inl.sum() and res.n_inliers <= inl.sum() + 3
    # an all-inlier sample scores the maximum possible for the inlier set
    assert res.score >= inl.sum() * float(vo.marginal_weight(0.0, 2.0)) * (1 - 1e-9)


def test_refinement_improves_noisy_estimates():
    gains = []
    for seed in range(6):
        a, b, H, inl = synth.homography_pairs(10 + seed, 400, outlier_frac=0.3, noise=0.7)
        u = synth.sample_numbers(20 + seed, 400)
        r0 = vo.verify(a, b, u, sigma_max=2.0, refine_iters=0)
        r1 = vo.verify(a, b, u, sigma_max=2.0, refine_iters=5)
        assert r1.score >= r0.score and r1.best == r0.best
        # distance of the estimate to the true model on the inliers' sources
        e0 = np.median(np.linalg.norm(vo.apply(r0.H, a[inl])[0] - vo.apply(H, a[inl])[0], axis=1))
        e1 = np.median(np.linalg.norm(vo.apply(r1.H, a[inl])[0] - vo.apply(H, a[inl])[0], axis=1))
        gains.append(e0 - e1)
    assert np.mean(gains) > 0


def test_degenerate_samples_give_no_hypothesis():
    a, b, H, _ = synth.homography_pairs(7, 40, outlier_frac=0.0, noise=0.0)
    u = np.zeros((3, 4), np.float32)
    u[0] = [0.1, 0.1, 0.5, 0.9]                     # repeated index
    a2 = a.copy()
    a2[:4] = [[0, 0], [10, 10], [20, 20], [30, 30]]  # collinear sources
    u[1] = [0.0, 0.025, 0.05, 0.075]                 # indices 0..3
    u[2] = [0.2, 0.4, 0.6, 0.8]
    res = vo.verify(a2, b, u, refine_iters=0)
    assert res.scores[0] == -np.inf and res.scores[1] == -np.inf
    assert np.isfinite(res.scores[2]) and res.best == 2


def test_order_of_correspondences_does_not_matter():
    a, b, H, _ = synth.homography_pairs(8, 200, outlier_frac=0.3, noise=0.3)
    u = synth.sample_numbers(9, 100)
    res = vo.verify(a, b, u)
    perm = np.random.default_rng(1).permutation(200)
    inv = np.argsort(perm)
    # the same samples, expressed in the permuted order: index i -> inv[i]
    idx = vo.sample_indices(u, 200)
    u2 = ((inv[idx] + 0.5) / 200).astype(np.float64)
    res2 = vo.verify(a[perm], b[perm], u2)
    assert res2.best == res.best
    np.testing.assert_allclose(res2.H, res.H, rtol=1e-9, atol=1e-9)
    assert res2.n_inliers == res.n_inliers


def test_too_few_correspondences():
    a, b, *_ = synth.homography_pairs(11, 3)
    res = vo.verify(a, b, synth.sample_numbers(1, 10))
    assert res.best == -1 and res.n_inliers == 0

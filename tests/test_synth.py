"""Seeded input generator: reproducible, in range, float32 (CPU)."""
import numpy as np

from paper_2605_17869_amd import synth


def test_same_seed_same_bytes_and_range():
    a = synth.blob_image(123, 60, 80, 30)
    b = synth.blob_image(123, 60, 80, 30)
    c = synth.blob_image(124, 60, 80, 30)
    assert a.dtype == np.float32 and a.shape == (60, 80)
    assert a.tobytes() == b.tobytes()
    assert a.tobytes() != c.tobytes()
    assert a.min() >= 0.0 and a.max() <= 1.0


def test_workload_recipes():
    w1 = synth.workload(1)
    assert w1.sizes == [(480, 640)] and w1.n_blobs == [200]
    assert w1.settings["n_octaves"] == 4 and w1.settings["upsample"] == 0
    w2 = synth.workload(2, 3)
    assert w2.sizes == [(768, 1024)] * 3 and w2.settings["upsample"] == 1
    w5 = synth.workload(5, 4)
    assert len(w5.settings["dsp_scales"]) == 10 and w5.settings["rootsift"] == 1
    assert all(400 <= h <= 900 and 600 <= w <= 1200 for h, w in w5.sizes)
    w4 = synth.workload(4, 5)
    assert w4.sizes == synth.workload(4, 7).sizes[:5]
    assert all(320 <= h <= 2048 and 320 <= w <= 2048 for h, w in w4.sizes)


def test_noise_level_and_blob_mean():
    img = synth.blob_image(5, 200, 200, 0).astype(np.float64)
    # pure low-passed noise around 0.5: std shrinks by the filter's gain
    assert abs(img.mean() - 0.5) < 2e-3
    assert 0.004 < img.std() < 0.012


def test_warped_copy_identity_parts():
    img = synth.blob_image(6, 64, 64, 10)
    out, fwd = synth.warped_copy(img, 99)
    assert out.shape == img.shape and out.dtype == np.float32
    lin = fwd[:, :2]
    s = np.sqrt(abs(np.linalg.det(lin)))
    assert 0.5 <= s <= 2.0
    assert np.allclose(lin / s, [[lin[0, 0] / s, -lin[1, 0] / s], [lin[1, 0] / s, lin[0, 0] / s]])


def test_poisson_arrivals_monotone():
    t = synth.poisson_arrivals(1, 1000, 50.0)
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 50.0) < 5.0

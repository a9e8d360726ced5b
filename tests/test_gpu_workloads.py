"""The larger workloads at their full image sizes, through the launch
configuration the benchmark uses (one batched call, or the server), against
the FP64 oracle on a sample of the images: the high-resolution mixed
orientation batch with affine-warped copies and a keypoint cap of 8192, the
DSP (10 domain sizes) + RootSIFT batch, and requests of random sizes served
by the continuous-batching server.  Needs an MI355X."""
import numpy as np
import pytest

import oracle
import parity
from oracle import sift_oracle as so
from paper_2605_17869_amd import synth
from gpu_util import digest, extract_batch, require_gpu, say
from test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu


def oracle_parity(img, settings, got, min_decisive):
    p = so.Params.from_settings(settings)
    ref = oracle.sift(img, p, keep_octaves=True)
    kp, desc, nf, nc = got
    return assert_parity(p, ref, kp, desc, nf, nc, min_decisive=min_decisive)


def test_highres_mixed_orientation_with_warped_copies():
    from paper_2605_17869_amd import Extractor
    wl = synth.workload(3, 4)              # 2 x 1066x1600 and 2 x 1600x1066
    orig = [wl.image(k) for k in range(len(wl.sizes))]
    warped = [synth.warped_copy(orig[k], synth.workload_seed(3, k, True))[0] for k in (0, 2)]
    batch = orig + warped
    ex = Extractor(wl.settings)
    res = extract_batch(ex, batch)
    for (kp, desc, nf, nc), im in zip(res, batch):
        assert len(kp) == min(nf, 8192)
        say(f"{im.shape}: {len(kp)} keypoints of {nf}")
    say("original 1066x1600 vs oracle")
    oracle_parity(batch[0], wl.settings, res[0], 500)
    say("warped copy of a 1600x1066 image vs oracle")
    oracle_parity(batch[5], wl.settings, res[5], 200)


def test_highres_image_capped_below_its_count():
    """A 1066x1600 image of the high-resolution workload with the keypoint cap
    set below its count: the kept keypoints are the oracle's first ones in
    canonical order."""
    from paper_2605_17869_amd import Extractor
    wl = synth.workload(3, 4)
    img = wl.image(0)
    p = so.Params.from_settings(wl.settings)
    ref = oracle.sift(img, p, keep_octaves=True)
    cap = ref.n_found // 2
    say(f"{img.shape}: oracle {ref.n_found} keypoints, cap {cap}")
    settings = dict(wl.settings, max_keypoints=cap)
    kp, desc, nf, nc = extract_batch(Extractor(settings), [img])[0]
    assert len(kp) == cap
    rep = parity.compare_capped(ref, kp, desc, p, so, cap)
    say(rep.summary())
    assert rep.ok, rep.mismatches[:5]
    assert rep.decisive_ok >= 300


def test_dsp_rootsift_batch():
    from paper_2605_17869_amd import Extractor
    wl = synth.workload(5, 6)
    assert wl.settings["rootsift"] == 1 and len(wl.settings["dsp_scales"]) == 10
    imgs = [wl.image(k) for k in range(len(wl.sizes))]
    ex = Extractor(wl.settings)
    res = extract_batch(ex, imgs)
    for k in (0, 3):
        say(f"image {k} {imgs[k].shape} vs oracle")
        oracle_parity(imgs[k], wl.settings, res[k], 100)
    # RootSIFT descriptors: non-negative, unit L2 norm
    desc = res[1][1]
    assert (desc >= 0).all()
    assert np.allclose(np.linalg.norm(desc, axis=1), 1.0, atol=1e-5)


def test_served_random_sizes_match_oracle():
    torch = require_gpu()
    from paper_2605_17869_amd import Extractor, Server
    wl = synth.workload(4, 40)
    # the most elongated and the largest of the first 40 request sizes, plus two others
    sizes = wl.sizes
    k_long = max(range(len(sizes)), key=lambda k: max(sizes[k]) / min(sizes[k]))
    k_big = max(range(len(sizes)), key=lambda k: sizes[k][0] * sizes[k][1])
    picks = [k_long, k_big, 0, 1]
    imgs = [wl.image(k) for k in picks]
    srv = Server(wl.settings, arena_bytes=4 << 30, max_batch=3, max_inflight=2)
    d = [torch.from_numpy(im).cuda() for im in imgs]
    torch.cuda.synchronize()
    tickets = [srv.submit(t) for t in d]
    got = [srv.wait(t)[1].host() for t in tickets]
    srv.close()
    ex = Extractor(wl.settings)
    alone = extract_batch(ex, imgs[:1])[0]
    assert digest(alone[0], alone[1]) == digest(got[0][0], got[0][1])
    for j in (0, 1):
        say(f"served {imgs[j].shape} vs oracle")
        oracle_parity(imgs[j], wl.settings, got[j], 150)

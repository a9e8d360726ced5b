"""Chained Gaussian levels (several levels of an octave in one launch) against
one launch per level: levels and features must be bit-identical for every
chain length, chunk height, storage mode and image shape, including images
smaller than a chain's halo, where every border row and column is computed
from mirrored data.  Needs an MI355X."""
import hashlib
import re

import numpy as np
import pytest

from paper_2605_17869_amd import synth
from gpu_util import digest, extract, extract_batch, require_gpu, say

pytestmark = pytest.mark.gpu

SIZES = [(97, 129), (480, 640), (333, 70), (53, 61), (56, 205), (64, 2500), (2100, 64)]


def run(settings, imgs):
    from paper_2605_17869_amd import Extractor
    ex = Extractor(settings)
    out = [digest(r[0], r[1]) + str(r[2:]) for r in extract_batch(ex, imgs)]
    p = ex.params
    n_oct = p.n_octaves + p.upsample
    for img in imgs[:3]:
        *_, ws = extract(ex, img, keep_ws=True)
        lv = [ex.level(ws, *img.shape, o - p.upsample, l).tobytes()
              for o in range(n_oct) for l in range(p.n_scales + 3)]
        out.append(hashlib.sha256(b"".join(lv)).hexdigest())
    return out


def launch_labels(settings, img):
    from paper_2605_17869_amd import Extractor, profile_launches, profile_start, profile_stop
    ex = Extractor(settings)
    profile_start()
    extract(ex, img)
    labels = [lab for stage, lab, *_ in profile_launches() if stage == "blur"]
    profile_stop()
    return labels


@pytest.mark.parametrize("up,fp16", [(1, 0), (0, 0), (1, 1), (0, 1)])
def test_chains_do_not_change_results(up, fp16):
    require_gpu()
    imgs = [synth.blob_image(700 + k, h, w, max(4, h * w // 800)) for k, (h, w) in enumerate(SIZES)]
    base = dict(synth.BASE_SETTINGS, n_octaves=3, upsample=up, pyramid_fp16=fp16)
    ref = run(dict(base, blur_chain=1), imgs)
    for chain in (2, 3, 4, 0):
        for rows in (32, 512):
            say(f"upsample={up} fp16={fp16} blur_chain={chain} tile_rows={rows}")
            assert run(dict(base, blur_chain=chain, tile_rows=rows), imgs) == ref


@pytest.mark.parametrize("up,fp16", [(1, 0), (0, 1)])
def test_detection_waves_do_not_change_results(up, fp16):
    """Four or eight waves per detection work-group share a band's column
    segments differently; candidates, keypoints and descriptors are the same."""
    require_gpu()
    imgs = [synth.blob_image(720 + k, h, w, max(4, h * w // 800)) for k, (h, w) in enumerate(SIZES)]
    base = dict(synth.BASE_SETTINGS, n_octaves=3, upsample=up, pyramid_fp16=fp16)
    from paper_2605_17869_amd import Extractor
    outs = {}
    for waves in (4, 8):
        say(f"upsample={up} fp16={fp16} detect_waves={waves}")
        ex = Extractor(dict(base, detect_waves=waves))
        outs[waves] = [digest(r[0], r[1]) + str(r[2:]) for r in extract_batch(ex, imgs)]
    assert outs[4] == outs[8]


def test_chains_are_launched():
    require_gpu()
    img = synth.blob_image(710, 300, 400, 100)
    st = dict(synth.BASE_SETTINGS, n_octaves=3, upsample=1)
    one = launch_labels(dict(st, blur_chain=1), img)
    three = launch_labels(dict(st, blur_chain=3), img)
    four = launch_labels(dict(st, blur_chain=4), img)
    say(f"one level per launch: {one}")
    say(f"up to 3 levels: {three}")
    say(f"up to 4 levels: {four}")
    # octave -1 (6 levels) and octaves 0, 1, 2 (levels 1..5)
    assert len(one) == 6 + 3 * 5 and not any(re.search(r"l\d+-", lab) for lab in one)
    # octave -1: (0, 1, 2) chained then 3, 4, 5; later octaves: (1, 2, 3) then 4, 5
    assert three[0].startswith("o-1 l0-2") and three[4].startswith("o0 l1-3")
    assert len(three) == 4 + 3 * 3
    assert four[0].startswith("o-1 l0-3") and len(four) == 3 + 3 * 3


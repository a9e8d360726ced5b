"""Replayable batches (sift_graph_*) and the chunk-height autotuner through
the C ABI.  Each replay re-reads the images in place: the test rewrites them
between replays, runs eager extractions in between, and checks every replay
against eager extraction bit for bit.  Needs an MI355X."""
import numpy as np
import pytest

from paper_2605_17869_amd import synth
from gpu_util import digest, extract, require_gpu, say

pytestmark = pytest.mark.gpu

SETTINGS = dict(synth.BASE_SETTINGS, n_octaves=3, upsample=1)
SIZES = [(120, 160), (200, 150), (96, 300)]


def images(seed):
    return [synth.blob_image(seed * 10 + k, h, w, max(1, int(h * w * 3 * synth.BLOB_DENSITY)))
            for k, (h, w) in enumerate(SIZES)]


def test_graph_replays_match_eager_extraction():
    torch = require_gpu()
    from paper_2605_17869_amd import Extractor
    ex = Extractor(SETTINGS)
    bufs = [torch.from_numpy(im).cuda() for im in images(1)]
    torch.cuda.synchronize()
    g = ex.graph(bufs)
    for rnd, seed in enumerate((1, 2, 3, 2)):
        new = images(seed)
        for b, im in zip(bufs, new):
            b.copy_(torch.from_numpy(im))
        ref = [extract(ex, im) for im in new]    # eager work between replays
        feats = g.launch()
        torch.cuda.synchronize()
        for k, f in enumerate(feats):
            kp, desc, nf, nc = f.host()
            assert digest(kp, desc) == digest(ref[k][0], ref[k][1]), (rnd, k)
            assert (nf, nc) == ref[k][2:], (rnd, k)
            if rnd == 0:
                assert len(kp) > 5
        say(f"replay {rnd} (seed {seed}) matches eager")
    g.close()


def test_autotune_picks_a_candidate():
    torch = require_gpu()
    from paper_2605_17869_amd import Extractor
    ex = Extractor(SETTINGS)
    bufs = [torch.from_numpy(im).cuda() for im in images(4)]
    torch.cuda.synchronize()
    best, ms = ex.autotune(bufs, warmup=1, reps=2)
    say(f"autotune: best {best}, {ms}")
    assert best in (64, 128, 256, 512)
    assert all(v > 0 for v in ms.values())
    assert ms[best] == min(ms.values())


def test_bucket_replays_images_of_other_sizes():
    """One bucket (4 slots, at most 220 x 320) serves launches of 3, then 4,
    then 1 images of sizes it was not recorded with; every result equals
    sift_extract on the image alone, bit for bit, with eager work between
    replays."""
    torch = require_gpu()
    from paper_2605_17869_amd import Extractor
    from paper_2605_17869_amd.sift import SiftError
    ex = Extractor(SETTINGS)
    bk = ex.bucket(4, 220, 320)
    rounds = [[(120, 160), (200, 150), (96, 300)],
              [(220, 320), (64, 64), (150, 200), (100, 250)],
              [(77, 91)]]
    for rnd, sizes in enumerate(rounds):
        imgs = [synth.blob_image(900 + 10 * rnd + k, h, w, max(1, int(h * w * 3 * synth.BLOB_DENSITY)))
                for k, (h, w) in enumerate(sizes)]
        ref = [extract(ex, im) for im in imgs]
        bufs = [torch.from_numpy(im).cuda() for im in imgs]
        feats = bk.launch(bufs)
        torch.cuda.synchronize()
        for k, f in enumerate(feats):
            kp, desc, nf, nc = f.host()
            assert digest(kp, desc) == digest(ref[k][0], ref[k][1]), (rnd, k)
            assert (nf, nc) == ref[k][2:], (rnd, k)
        say(f"bucket round {rnd}: {len(sizes)} images match sift_extract")
    big = torch.zeros((221, 100), dtype=torch.float32, device="cuda")
    with pytest.raises(SiftError):
        bk.launch([big])
    five = [torch.full((100, 100), 0.5, dtype=torch.float32, device="cuda")] * 5
    with pytest.raises(SiftError):
        bk.launch(five)
    bk.close()


def test_bucket_needs_one_octave_structure():
    torch = require_gpu()
    from paper_2605_17869_amd import Extractor
    from paper_2605_17869_amd.sift import SiftError
    ex = Extractor(dict(SETTINGS, upsample_max_pixels=20000))
    bk = ex.bucket(2, 200, 200)            # 40000 px: built without octave -1
    small = torch.full((100, 150), 0.5, dtype=torch.float32, device="cuda")   # 15000 px: upsampled
    with pytest.raises(SiftError):
        bk.launch([small])
    img = synth.blob_image(950, 180, 190, 60)
    ref = extract(ex, img)
    f, = bk.launch([torch.from_numpy(img).cuda()])
    torch.cuda.synchronize()
    kp, desc, nf, nc = f.host()
    assert digest(kp, desc) == digest(ref[0], ref[1])
    bk.close()


def test_tuning_cache_round_trip(tmp_path):
    """sift_autotune times the launch knobs, appends the winner to the cache file,
    and a second call with the same batch reads it back without timing; the
    tuned handle gives the same bits as any other setting."""
    torch = require_gpu()
    from paper_2605_17869_amd import Extractor
    ex = Extractor(SETTINGS)
    imgs = images(6)
    bufs = [torch.from_numpy(im).cuda() for im in imgs]
    cache = str(tmp_path / "tune.txt")
    first = ex.tune(bufs, warmup=1, reps=1, cache_path=cache)
    say(f"tuned: {first}")
    assert not first["from_cache"] and first["candidates_timed"] >= 4
    assert first["tile_rows"] in (64, 128, 256, 512) and first["n_streams"] in (1, 2)
    assert first["blur_chain"] in (1, 2, 3) and first["detect_waves"] in (4, 8)
    again = ex.tune(bufs, warmup=1, reps=1, cache_path=cache)
    assert again["from_cache"] and again["candidates_timed"] == 0
    knobs = lambda t: (t["tile_rows"], t["n_streams"], t["blur_chain"], t["detect_waves"])
    assert knobs(again) == knobs(first)
    graph = ex.tune(bufs, warmup=1, reps=1, cache_path=cache, as_graph=True)
    assert not graph["from_cache"] and graph["candidates_timed"] >= 4   # its own key
    assert ex.tune(bufs, warmup=1, reps=1, cache_path=cache, as_graph=True)["from_cache"]
    tuned = Extractor(dict(SETTINGS, tile_rows=first["tile_rows"], n_streams=first["n_streams"],
                           blur_chain=first["blur_chain"], detect_waves=first["detect_waves"]))
    ref = [extract(ex, im) for im in imgs]
    feats = tuned.extract_batch(bufs)
    torch.cuda.synchronize()
    for k, f in enumerate(feats):
        kp, desc, nf, nc = f.host()
        assert digest(kp, desc) == digest(ref[k][0], ref[k][1])

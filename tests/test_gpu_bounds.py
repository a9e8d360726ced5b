"""The kernels built with bounds checks (libsift_mi355x_bounds.so) on shapes
and settings that reach the edges of the index arithmetic: images smaller
than a chained launch's halo, one strip wide or tall, ragged chunks, fp16
storage, the upsampled octave, pooled descriptor sizes, five scales per
octave, a keypoint cap, sub-batches.  No checked access may leave the memory
it belongs to, and the results must be those of the normal library bit for
bit.  Needs an MI355X."""
import pytest

from paper_2605_17869_amd import synth
from gpu_util import digest, extract, extract_batch, require_gpu, say

pytestmark = pytest.mark.gpu

SIZES = [(97, 129), (53, 61), (56, 205), (64, 2500), (2100, 64), (480, 640), (333, 70)]

CASES = [
    ("upsampled", dict(upsample=1)),
    ("fp16 storage", dict(pyramid_fp16=1)),
    ("one level per launch, 32-row chunks", dict(upsample=1, blur_chain=1, tile_rows=32)),
    ("three levels per launch, 8 detection waves", dict(blur_chain=3, detect_waves=8)),
    ("pooled sizes, RootSIFT", dict(dsp_scales=list(synth.dsp_linspace()), rootsift=1)),
    ("five scales per octave", dict(n_scales=5)),
    ("keypoint cap", dict(max_keypoints=50, max_candidates=200)),
]


@pytest.mark.parametrize("name,over", CASES, ids=[c[0] for c in CASES])
def test_no_access_out_of_bounds(name, over):
    require_gpu()
    from paper_2605_17869_amd import Extractor, bounds_violations
    imgs = [synth.blob_image(900 + k, h, w, max(4, h * w // 800)) for k, (h, w) in enumerate(SIZES)]
    imgs += imgs[:3]   # ten images: the batch runs as sub-batches
    settings = dict(synth.BASE_SETTINGS, n_octaves=3, **over)
    say(f"bounds-checked extraction: {name}")
    bounds_violations(reset=True)
    ref = [digest(r[0], r[1]) + str(r[2:]) for r in extract_batch(Extractor(settings), imgs)]
    checked = Extractor(settings, bounds_checked=True)
    got = [digest(r[0], r[1]) + str(r[2:]) for r in extract_batch(checked, imgs)]
    n = bounds_violations(reset=True)
    say(f"{name}: {n} out-of-range accesses")
    assert n == 0
    assert got == ref


def test_matcher_and_verifier_in_bounds():
    """Matching (ragged row tiles, device counts below capacity, single rows)
    and verification (counts below capacity, too few correspondences) on the
    bounds-checked library: no access out of range, the same bits."""
    import numpy as np
    torch = require_gpu()
    from paper_2605_17869_amd import bounds_violations, match_batch, verify_batch

    sets = [synth.descriptor_sets(s, na, nb, nc, 0.12)[:2]
            for s, na, nb, nc in [(950, 129, 257, 100), (951, 1, 5, 1), (952, 700, 600, 400)]]
    counts = [None, None, (450, 333)]

    def matches(bounds):
        args = []
        for (a, b), c in zip(sets, counts):
            ta = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
            tb = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float32)).cuda()
            ca = cb = None
            if c is not None:
                ca = torch.tensor([c[0]], dtype=torch.int32, device="cuda")
                cb = torch.tensor([c[1]], dtype=torch.int32, device="cuda")
            args.append((ta, ca, tb, cb))
        out = match_batch(args, bounds_checked=bounds)
        torch.cuda.synchronize()
        return [(m.host()[0].tobytes(), m.host()[1]) for m in out]

    def verified(bounds):
        pairs = []
        for seed, n, cnt in [(960, 500, 321), (961, 300, None), (962, 3, None)]:
            a, b, _, _ = synth.homography_pairs(seed, n, 0.3, 0.5)
            ka = np.zeros((n, 12), np.int32)
            kb = np.zeros((n, 12), np.int32)
            ka.view(np.float32)[:, 0:2] = a.astype(np.float32)
            kb.view(np.float32)[:, 0:2] = b.astype(np.float32)
            m = np.zeros((n, 4), np.int32)
            m[:, 0] = np.arange(n)
            m[:, 1] = np.arange(n)
            c = None if cnt is None else torch.tensor([cnt], dtype=torch.int32, device="cuda")
            pairs.append((torch.from_numpy(ka).cuda(), torch.from_numpy(kb).cuda(),
                          torch.from_numpy(m).cuda(), c))
        u = torch.from_numpy(synth.sample_numbers(963, 1500)).cuda()
        out = verify_batch(pairs, u, bounds_checked=bounds)
        torch.cuda.synchronize()
        return [repr([np.asarray(x).tobytes() if isinstance(x, np.ndarray) else x
                      for x in r.host()]) for r in out]

    say("bounds-checked matching and verification")
    bounds_violations(reset=True)
    assert matches(True) == matches(False)
    assert verified(True) == verified(False)
    n = bounds_violations(reset=True)
    say(f"matching and verification: {n} out-of-range accesses")
    assert n == 0


def test_batch_beyond_the_lds_prefix_tables():
    """One sub-batch of 1,030 small images: more than the orientation and
    descriptor kernels keep of the batch's prefix tables in LDS, so both search
    them in global memory.  Every image's results equal those of extracting it
    alone, and the bounds-checked library finds nothing out of range."""
    require_gpu()
    from paper_2605_17869_amd import Extractor, bounds_violations
    sizes = [(64 + (k % 5) * 8, 64 + (k % 7) * 8) for k in range(1030)]
    imgs = [synth.blob_image(5000 + k, h, w, 6) for k, (h, w) in enumerate(sizes)]
    settings = dict(synth.BASE_SETTINGS, n_octaves=2, max_keypoints=256, max_candidates=256,
                    n_streams=1)
    say(f"{len(imgs)} images in one launch sequence")
    batch = [digest(r[0], r[1]) + str(r[2:]) for r in extract_batch(Extractor(settings), imgs)]
    ex = Extractor(settings)
    alone = []
    for im in imgs[::103]:
        kp, desc, nf, nc = extract(ex, im)
        alone.append(digest(kp, desc) + str((nf, nc)))
    assert alone == batch[::103]
    bounds_violations(reset=True)
    checked = [digest(r[0], r[1]) + str(r[2:])
               for r in extract_batch(Extractor(settings, bounds_checked=True), imgs)]
    n = bounds_violations(reset=True)
    say(f"1,030 images: {n} out-of-range accesses")
    assert n == 0 and checked == batch

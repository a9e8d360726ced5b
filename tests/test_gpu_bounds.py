"""The kernels built with bounds checks (libsift_mi355x_bounds.so) on shapes
and settings that reach the edges of the index arithmetic: images smaller
than a chained launch's halo, one strip wide or tall, ragged chunks, fp16
storage, the upsampled octave, pooled descriptor sizes, five scales per
octave, a keypoint cap, sub-batches.  No checked access may leave the memory
it belongs to, and the results must be those of the normal library bit for
bit.  Needs an MI355X."""
import pytest

from paper_2605_17869_amd import synth
from gpu_util import digest, extract_batch, require_gpu, say

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

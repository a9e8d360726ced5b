"""sift_extract_noalloc (the entry point that allocates nothing: its workspace
is the library's static device scratch) against sift_extract on the same
images, through the C ABI: two calls in a row, the second on a smaller image,
must give the same bits as the workspace-taking entry point.  Needs an MI355X."""
import numpy as np
import pytest

from paper_2605_17869_amd import synth
from gpu_util import require_gpu, say

pytestmark = pytest.mark.gpu


def _features_equal(a, b):
    ka, da, nfa, nca = a
    kb, db, nfb, ncb = b
    assert (nfa, nca) == (nfb, ncb)
    assert ka.shape == kb.shape
    assert ka.tobytes() == kb.tobytes()
    assert np.array_equal(da.view(np.uint32), db.view(np.uint32))


def test_noalloc_matches_extract_on_two_calls():
    torch = require_gpu()
    from paper_2605_17869_amd import Extractor
    from paper_2605_17869_amd.sift import load_library
    lib = load_library()
    assert lib.sift_noalloc_scratch_bytes() == 64 << 20
    settings = dict(synth.BASE_SETTINGS)
    ex = Extractor(settings)
    # first a larger image, then a smaller one: the second call must not see
    # anything the first left in the shared scratch
    sizes = [(768, 1024, 1000), (480, 640, 200)]
    for i, (h, w, nb) in enumerate(sizes):
        img = synth.blob_image(7100 + i, h, w, nb)
        say(f"noalloc call {i}: {h}x{w}, workspace {ex.workspace_size(h, w)} bytes")
        t = torch.from_numpy(img).cuda()
        ref = ex.extract(t)                      # workspace-taking entry point
        torch.cuda.synchronize()
        ref_h = ref.host()
        out = ex.alloc_features()
        ex.extract_noalloc(t, out)
        torch.cuda.synchronize()
        got = out.host()
        say(f"  {len(got[0])} keypoints, n_found {got[2]}, candidates {got[3]}")
        assert len(got[0]) > 50
        _features_equal(ref_h, got)


def test_noalloc_rejects_images_beyond_scratch():
    torch = require_gpu()
    from paper_2605_17869_amd import Extractor
    from paper_2605_17869_amd.sift import SiftError
    ex = Extractor(dict(synth.BASE_SETTINGS))
    h, w = 2048, 2048
    assert ex.workspace_size(h, w) > 64 << 20
    t = torch.full((h, w), 0.5, dtype=torch.float32, device="cuda")
    out = ex.alloc_features()
    with pytest.raises(SiftError) as ei:
        ex.extract_noalloc(t, out)
    assert ei.value.status == 3   # SIFT_ERR_WORKSPACE_TOO_SMALL, nothing enqueued
    assert "static scratch" in str(ei.value)
    # the entry point still works after the refusal
    img = synth.blob_image(7200, 480, 640, 200)
    small = torch.from_numpy(img).cuda()
    ex.extract_noalloc(small, out)
    ref = ex.extract(small)
    torch.cuda.synchronize()
    _features_equal(ref.host(), out.host())

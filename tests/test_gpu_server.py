"""The continuous-batching server (sift_server_* through the C ABI): every
request's outputs equal a plain sift_extract of the same image bit for bit,
whatever batches and streams the requests landed in; admission respects the
arena; oversize requests are refused.  Needs an MI355X."""
import numpy as np
import pytest

from paper_2605_17869_amd import synth
from gpu_util import digest, extract, require_gpu, say

pytestmark = pytest.mark.gpu

SETTINGS = dict(synth.BASE_SETTINGS, n_octaves=3, max_candidates=4096, max_keypoints=2048)


def requests(seed, n):
    rng = np.random.default_rng(seed)
    sizes = [(int(rng.integers(90, 420)), int(rng.integers(90, 420))) for _ in range(n)]
    return [synth.blob_image(seed * 100 + k, h, w, max(1, int(h * w * 3 * synth.BLOB_DENSITY)))
            for k, (h, w) in enumerate(sizes)]


def serve(imgs, arena_bytes, max_batch, max_inflight, group=False):
    torch = require_gpu()
    from paper_2605_17869_amd import Server
    srv = Server(SETTINGS, arena_bytes=arena_bytes, max_batch=max_batch,
                 max_inflight=max_inflight)
    d = [torch.from_numpy(im).cuda() for im in imgs]
    torch.cuda.synchronize()
    tickets = srv.submit_many(d) if group else [srv.submit(t) for t in d]
    results = []
    for t in tickets:
        lat, f = srv.wait(t)
        assert lat >= 0.0
        results.append(f.host())
    stats = srv.stats()
    srv.close()
    return results, stats


def test_served_outputs_equal_plain_extraction():
    from paper_2605_17869_amd import Extractor
    imgs = requests(5, 14)
    ex = Extractor(SETTINGS)
    ref = [extract(ex, im) for im in imgs]
    one = max(ex.workspace_size(*im.shape) for im in imgs)
    # room for about three of the largest images at once: batches are cut by
    # footprint; with room for all, batches of 8 or more images form, which
    # the batched call runs as sub-batches with a header each
    small, large = 3 * one + (1 << 20), 16 * one
    for max_batch, max_inflight, arena, group in ((4, 2, small, False), (1, 1, small, False),
                                                  (64, 3, small, False), (64, 1, large, True),
                                                  (12, 2, large, True), (64, 2, large, False)):
        say(f"max_batch={max_batch} max_inflight={max_inflight} arena={arena} group={group}")
        got, stats = serve(imgs, arena, max_batch, max_inflight, group)
        say(f"  stats {stats}")
        assert stats["submitted"] == stats["completed"] == len(imgs)
        assert stats["peak_arena"] <= arena
        assert stats["peak_inflight"] <= max_inflight
        assert stats["largest_batch"] <= max_batch
        if max_batch == 1:
            assert stats["batches"] == len(imgs)
        if group:
            # the whole group reaches an idle worker at once: with room for
            # all, the first batch takes min(max_batch, 14) requests, a batch
            # of 8 or more that the batched call splits into sub-batches
            assert stats["largest_batch"] == min(max_batch, len(imgs)) >= 8
        for k, (a, b) in enumerate(zip(ref, got)):
            assert digest(a[0], a[1]) == digest(b[0], b[1]), k
            assert a[2:] == b[2:], k


def test_oversize_request_is_refused():
    torch = require_gpu()
    from paper_2605_17869_amd import Extractor, Server, SiftError
    ex = Extractor(SETTINGS)
    small = requests(9, 1)[0]
    srv = Server(SETTINGS, arena_bytes=ex.workspace_size(*small.shape) + 4096, max_batch=4,
                 max_inflight=1)
    big = torch.zeros((1500, 1500), dtype=torch.float32, device="cuda")
    with pytest.raises(SiftError) as ei:
        srv.submit(big)
    assert ei.value.status == 4
    # the server still serves what fits
    d_small = torch.from_numpy(small).cuda()
    torch.cuda.synchronize()
    t = srv.submit(d_small)
    lat, f = srv.wait(t)
    kp, desc, nf, nc = f.host()
    ref = extract(ex, small)
    assert digest(kp, desc) == digest(ref[0], ref[1])
    srv.close()

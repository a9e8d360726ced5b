"""The parity checker itself (CPU only): the oracle's own output passes, and a
reordered, truncated or wrongly capped output fails."""
import numpy as np

import oracle
import parity
from oracle import sift_oracle as so
from paper_2605_17869_amd import synth


def oracle_run(**kw):
    p = so.Params(n_octaves=3, **kw)
    img = synth.blob_image(21, 120, 150, 90)
    return p, oracle.sift(img, p, keep_octaves=True)


def test_oracle_output_passes_and_reordering_fails():
    p, ref = oracle_run()
    kps, desc = ref.keypoints, ref.descriptors
    assert len(kps) > 20
    rep = parity.compare(ref, kps, desc, p, so)
    assert rep.ok, rep.mismatches[:3]
    assert rep.decisive_ok > 10
    # swap two keypoints of different detections: same set, wrong order
    keys = parity.source_keys(kps)
    j = next(k for k in range(1, len(keys)) if keys[k] != keys[0])
    perm = np.arange(len(kps))
    perm[[0, j]] = perm[[j, 0]]
    bad = parity.compare(ref, kps[perm], desc[perm], p, so)
    assert not bad.ok
    assert any("order" in m[1] for m in bad.mismatches)
    # drop one keypoint of a decisive detection
    drop = parity.compare(ref, np.delete(kps, 3), np.delete(desc, 3, axis=0), p, so)
    assert not drop.ok


def test_capped_output_against_the_full_oracle():
    p, ref = oracle_run()
    cap = len(ref.keypoints) // 2
    pc, capped = oracle_run(max_keypoints=cap)
    assert len(capped.keypoints) == cap and capped.n_found == ref.n_found
    rep = parity.compare_capped(ref, capped.keypoints, capped.descriptors, p, so, cap)
    assert rep.ok, rep.mismatches[:3]
    # a prefix one short of the cap, or the wrong window of the sequence, fails
    short = parity.compare_capped(ref, ref.keypoints[:cap - 1], ref.descriptors[:cap - 1], p,
                                  so, cap)
    assert not short.ok
    shifted = parity.compare_capped(ref, ref.keypoints[1:cap + 1], ref.descriptors[1:cap + 1],
                                    p, so, cap)
    assert not shifted.ok

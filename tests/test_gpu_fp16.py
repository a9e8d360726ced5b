"""fp16 pyramid storage (pyramid_fp16 = 1; section 3.2, "GPU Pipeline Stages":
fp16 storage, fp32 compute, the first octave in fp32) against the oracle's
fp16-storage mode.  Needs an MI355X.

Tolerances for the octaves stored in fp16 are restated from the arithmetic:
the kernels round an fp32 blur result to fp16 and the oracle an fp64 one, so
a stored value can differ by one fp16 ulp where the two straddle a rounding
boundary (2^-12 for |L - 1/2| in [1/4, 1/2)).  Two such levels make a DoG
error of up to ~5e-4, against a pre-gate of 0.0067 and a contrast threshold
of 0.0133; the sub-pixel offset moves by the DoG error over the Hessian,
under 0.05 octave pixels, i.e. 0.05 * 2^o input pixels; angles by under 1
degree and descriptors by under 2e-2 over many samples.  The first octave
is stored in fp32 and keeps the fp32 bar unchanged."""
import numpy as np
import pytest

import oracle
import parity
from oracle import sift_oracle as so
from paper_2605_17869_amd import synth
from gpu_util import digest, extract, extract_batch, require_gpu, say

pytestmark = pytest.mark.gpu

FP16_ULP = 2.0 ** -12


def settings16(**kw):
    return dict(synth.BASE_SETTINGS, pyramid_fp16=1, **kw)


@pytest.mark.parametrize("up", [0, 1])
def test_fp16_levels_match_oracle(up):
    from paper_2605_17869_amd import Extractor
    st = settings16(upsample=up, n_octaves=3)
    img = synth.blob_image(61, 150, 190, 60)
    p = so.Params.from_settings(st)
    octs = so.scale_space(img, p)
    ex = Extractor(st)
    *_, ws = extract(ex, img, keep_ws=True)
    for j, oc in enumerate(octs):
        for lv in range(p.n_scales + 3):
            g = ex.level(ws, img.shape[0], img.shape[1], oc.o, lv)
            d = np.abs(g - oc.L[lv])
            if j == 0:
                assert d.max() < 2e-6, (oc.o, lv, d.max())
            else:
                # fp16 values (centred), apart by at most a couple of ulps at the
                # few pixels where the fp32 and fp64 results round differently
                centred = g - 0.5
                assert np.array_equal(centred, centred.astype(np.float16).astype(np.float64))
                assert d.max() <= 2 * FP16_ULP, (oc.o, lv, d.max())
                assert np.mean(d > 0) < 0.05, (oc.o, lv, np.mean(d > 0))
    say(f"upsample={up}: fp16 levels within {2 * FP16_ULP:.2g} of the oracle's")


def test_fp16_keypoints_match_oracle():
    """First octave (fp32 storage): the fp32 bar.  Octaves stored in fp16: a
    candidate whose neighbour gaps are below the fp16 rounding noise of its
    levels is decided by that noise on either side, and about half are (their
    extremum margin is ~1e-2 against a noise of ~2 ulps / |D|), so the bar is an
    agreement rate: at least 90 % of the oracle's keypoints there have a GPU
    keypoint from the same detection at the same integer (layer, row, col),
    those agree within the restated tolerances, and at most 10 % of the GPU's
    keypoints there have no oracle counterpart."""
    wl = synth.workload(1)
    img = wl.image(0)
    st = settings16()
    from paper_2605_17869_amd import Extractor
    p = so.Params.from_settings(st)
    ref = oracle.sift(img, p, keep_octaves=True)
    kp, desc, nf, nc = extract(Extractor(st), img)
    first = {(e["o"], e["i0"], e["r0"], e["c0"]) for e in ref.log if e["o"] == 0}
    rep = parity.compare(ref, kp[kp["octave"] == 0], desc[kp["octave"] == 0], p, so,
                         sample=first)
    say(f"first octave (fp32 storage): {rep.summary()}")
    assert rep.ok and rep.decisive_ok > 20
    gpu = parity.group_by_source(kp)
    ref_n = matched = 0
    worst = dict(xy=0.0, angle=0.0, desc=0.0)
    for e in ref.log:
        if e["o"] == 0 or e["status"] != "ok":
            continue
        ref_n += len(e["angles"])
        rows = gpu.get((e["o"], e["i0"], e["r0"], e["c0"]), [])
        if len(rows) != len(e["angles"]) or any(
                (int(kp["layer"][r]), int(kp["iy"][r]), int(kp["ix"][r])) != (e["i"], e["r"], e["c"])
                for r in rows):
            continue
        for k, r in enumerate(rows):
            exy = max(abs(float(kp["x"][r]) - e["x"]), abs(float(kp["y"][r]) - e["y"]))
            ea = float(parity.angle_diff(kp["angle"][r], e["angles"][k]))
            ed = float(np.max(np.abs(desc[r].astype(np.float64) - e["desc"][k])))
            assert exy <= 0.05 * 2.0 ** e["o"], (e["o"], exy)
            assert ea <= 1.0 and ed <= 2e-2, (ea, ed)
            worst = {kk: max(worst[kk], v) for kk, v in zip(("xy", "angle", "desc"), (exy, ea, ed))}
            matched += 1
    gpu_n = int(np.sum(kp["octave"] > 0))
    say(f"fp16 octaves: oracle {ref_n} keypoints, GPU {gpu_n}, matched {matched}; worst {worst}")
    assert ref_n > 50
    assert matched >= 0.9 * ref_n
    assert gpu_n - matched <= 0.1 * gpu_n


def test_fp16_first_octave_equals_fp32_storage():
    """Storage of the later octaves does not touch the first octave's
    keypoints: bit-identical between the two modes."""
    from paper_2605_17869_amd import Extractor
    img = synth.workload(1).image(0)
    k32, d32, _, _ = extract(Extractor(dict(synth.BASE_SETTINGS)), img)
    k16, d16, _, _ = extract(Extractor(settings16()), img)
    s32, s16 = k32["octave"] == 0, k16["octave"] == 0
    assert s32.sum() > 20
    assert k32[s32].tobytes() == k16[s16].tobytes()
    assert d32[s32].tobytes() == d16[s16].tobytes()


def test_fp16_batch_equals_single_and_dsp():
    from paper_2605_17869_amd import Extractor
    st = settings16(upsample=1, n_octaves=4, dsp_scales=synth.dsp_linspace(), rootsift=1)
    imgs = [synth.blob_image(70 + k, h, w, int(h * w * synth.BLOB_DENSITY))
            for k, (h, w) in enumerate([(300, 400), (257, 333), (400, 300)])]
    ex = Extractor(st)
    batch = extract_batch(ex, imgs)
    for k, im in enumerate(imgs):
        one = extract(ex, im)
        assert digest(one[0], one[1]) == digest(batch[k][0], batch[k][1])
        assert len(one[0]) > 10

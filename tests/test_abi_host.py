"""C ABI on the host: the library loads, exports every declared entry point,
its structs match the binding, and argument errors come back before any GPU
work (CPU only: no call here reaches a kernel)."""
import ctypes
import re
import subprocess
from pathlib import Path

import pytest

from paper_2605_17869_amd import sift as S

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "sift.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sift_[a-z_]+)\s*\(", text)))


@pytest.mark.parametrize("bounds", [False, True])
def test_library_exports_every_declared_symbol(bounds):
    """Both libraries: the normal one and its bounds-checked twin."""
    lib = S.load_library(bounds=bounds)
    names = declared_functions()
    assert "sift_extract" in names and "sift_extract_batch" in names and "sift_create" in names
    for name in names:
        assert hasattr(lib, name), name
    path = S.BOUNDS_LIB_PATH if bounds else S.LIB_PATH
    nm = subprocess.run(["nm", "-D", "--defined-only", str(path)], capture_output=True,
                        text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sift_\w+)", nm))
    assert set(names) <= exported


def test_bounds_query_of_the_normal_library():
    """The normal library has no bounds checks: it says so before any device call."""
    lib = S.load_library()
    n = ctypes.c_uint64(7)
    assert lib.sift_bounds_violations(1, ctypes.byref(n)) == 6 and n.value == 0   # NOT_SUPPORTED
    assert b"bounds" in lib.sift_last_error()
    assert lib.sift_bounds_violations(0, None) == 1                               # INVALID_ARG
    assert S.load_library(bounds=True).sift_bounds_violations(0, None) == 1


PROBE = r"""
#include <stdio.h>
#include <stddef.h>
#include "sift.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m))
int main(void) {
  printf("sift_params %zu\nsift_keypoint %zu\nsift_output %zu\nsift_stage_stat %zu\n",
         sizeof(sift_params), sizeof(sift_keypoint), sizeof(sift_output), sizeof(sift_stage_stat));
  printf("sift_server_stats %zu\n", sizeof(sift_server_stats));
  F(sift_server_stats, largest_batch); F(sift_server_stats, overlapped_batches);
  F(sift_params, dsp_scales); F(sift_params, rootsift); F(sift_params, max_candidates);
  F(sift_keypoint, octave); F(sift_keypoint, src_ix);
  F(sift_output, n_candidates); F(sift_output, capacity);
  F(sift_stage_stat, ms); F(sift_stage_stat, bytes);
  return 0;
}
"""


def test_struct_layouts_match_the_binding(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(PROBE)
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", str(ROOT / "include"), str(src), "-o", str(exe)],
                   check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True,
                                                       text=True, check=True).stdout.splitlines())
    assert int(out["sift_params"]) == ctypes.sizeof(S.SiftParams)
    assert int(out["sift_keypoint"]) == S.KEYPOINT_DTYPE.itemsize == 48
    assert int(out["sift_output"]) == ctypes.sizeof(S.SiftOutput)
    assert int(out["sift_stage_stat"]) == ctypes.sizeof(S.SiftStageStat)
    assert int(out["sift_server_stats"]) == ctypes.sizeof(S.SiftServerStats)
    for key, val in out.items():
        if "." not in key:
            continue
        t, m = key.split(".")
        cls = {"sift_params": S.SiftParams, "sift_output": S.SiftOutput,
               "sift_stage_stat": S.SiftStageStat, "sift_server_stats": S.SiftServerStats}.get(t)
        if cls is not None:
            assert getattr(cls, m).offset == int(val), key
        else:
            assert S.KEYPOINT_DTYPE.fields[m][1] == int(val), key


def test_defaults_and_parameter_validation():
    p = S.make_params()
    assert (p.n_octaves, p.n_scales, p.upsample, p.ori_bins, p.desc_width) == (4, 3, 0, 36, 4)
    assert abs(p.contrast_threshold - 0.04 / 3) < 1e-8 and p.n_dsp == 1
    lib = S.load_library()
    h = ctypes.c_void_p()
    for bad, code in [(dict(n_scales=0), 6), (dict(n_scales=7), 6), (dict(ori_bins=32), 6),
                      (dict(border=0), 1), (dict(desc_width=3), 6), (dict(upsample=2), 1),
                      (dict(n_octaves=12, upsample=1), 6), (dict(sigma0=9.0), 6),
                      (dict(max_candidates=0), 1), (dict(ori_peak_ratio=1.5), 1),
                      (dict(tile_rows=48), 1), (dict(tile_rows=1024), 1), (dict(n_streams=9), 1),
                      (dict(blur_chain=-1), 1), (dict(blur_chain=5), 1),
                      (dict(detect_waves=2), 1), (dict(detect_waves=16), 1),
                      (dict(detect_waves=-4), 1)]:
        pp = S.make_params(**bad)
        assert lib.sift_create(ctypes.byref(pp), ctypes.byref(h)) == code, bad
        assert lib.sift_last_error()
    for rows in (0, 32, 64, 128, 256, 512):
        S.Extractor(tile_rows=rows)
    for chain in range(5):
        S.Extractor(blur_chain=chain)
    for waves in (0, 4, 8):
        S.Extractor(detect_waves=waves)
    with pytest.raises(S.SiftError):
        S.Extractor(n_scales=0)
    ex = S.Extractor(dsp_scales=[0.5, 1.0, 2.0], rootsift=1)
    q = S.SiftParams()
    assert lib.sift_get_params(ex.handle, ctypes.byref(q)) == 0
    assert q.n_dsp == 3 and q.rootsift == 1 and abs(q.dsp_scales[2] - 2.0) < 1e-7


def test_workspace_size_rules():
    ex = S.Extractor()
    n = ex.workspace_size(480, 640)
    # at least the pyramid: 6 levels of every octave, fp32
    assert n > 6 * 4 * (480 * 640 + 240 * 320 + 120 * 160 + 60 * 80)
    assert ex.workspace_size(481, 641) >= n
    with pytest.raises(S.SiftError) as ei:
        ex.workspace_size(100, 100)          # last octave 13x13 needs >= 13: ok
        ex.workspace_size(96, 100)           # 12 rows at octave 3
    assert ei.value.status == 2
    with pytest.raises(S.SiftError) as ei:
        ex.workspace_size(0, 100)
    assert ei.value.status == 1
    with pytest.raises(S.SiftError) as ei:
        ex.workspace_size(40000, 100)
    assert ei.value.status == 4
    with pytest.raises(S.SiftError) as ei:     # a 3.6 GB level
        ex.workspace_size(30000, 30000)
    assert ei.value.status == 4
    assert S.Extractor(upsample=1).workspace_size(11000, 11000) > 0
    up = S.Extractor(upsample=1)
    assert up.workspace_size(480, 640) > 2 * n
    b = ex.batch_workspace_size([(480, 640), (300, 200)])
    assert b > n


def test_extract_argument_errors_return_before_any_launch():
    lib = S.load_library()
    ex = S.Extractor()
    out = S.SiftOutput(1024, 2048, 4096, 0, 0, 10)
    stream = ctypes.c_void_p()
    # null image
    st = lib.sift_extract(ex.handle, None, 480, 640, 640, ctypes.c_void_p(256), 1 << 30,
                          ctypes.byref(out), stream)
    assert st == 1
    # pitch below width
    st = lib.sift_extract(ex.handle, ctypes.c_void_p(512), 480, 640, 600, ctypes.c_void_p(256),
                          1 << 30, ctypes.byref(out), stream)
    assert st == 1
    # misaligned workspace
    st = lib.sift_extract(ex.handle, ctypes.c_void_p(512), 480, 640, 640, ctypes.c_void_p(260),
                          1 << 30, ctypes.byref(out), stream)
    assert st == 1
    # workspace too small
    st = lib.sift_extract(ex.handle, ctypes.c_void_p(512), 480, 640, 640, ctypes.c_void_p(256),
                          1024, ctypes.byref(out), stream)
    assert st == 3
    # image too small for the octave count
    st = lib.sift_extract(ex.handle, ctypes.c_void_p(512), 50, 640, 640, ctypes.c_void_p(256),
                          1 << 30, ctypes.byref(out), stream)
    assert st == 2
    # null output pointers
    bad = S.SiftOutput(0, 2048, 4096, 0, 0, 10)
    st = lib.sift_extract(ex.handle, ctypes.c_void_p(512), 480, 640, 640, ctypes.c_void_p(256),
                          1 << 30, ctypes.byref(bad), stream)
    assert st == 1
    # empty batch
    st = lib.sift_extract_batch(ex.handle, 0, None, None, None, None, ctypes.c_void_p(256),
                                1 << 30, None, stream)
    assert st == 1


def test_status_strings_and_profile_misuse():
    lib = S.load_library()
    assert lib.sift_status_string(0) == b"ok"
    assert lib.sift_status_string(3) == b"workspace too small"
    arr = (S.SiftStageStat * 4)()
    n = ctypes.c_int32()
    assert lib.sift_profile_stop(arr, 4, ctypes.byref(n)) == 1
    assert lib.sift_profile_start() == 0
    assert lib.sift_profile_stop(arr, 4, ctypes.byref(n)) == 0 and n.value == 0


def test_server_argument_errors_return_before_any_device_call():
    lib = S.load_library()
    p = S.make_params()
    srv = ctypes.c_void_p()
    # null arena, misaligned arena, batch and in-flight limits
    assert lib.sift_server_create(ctypes.byref(p), None, 1 << 30, 8, 2, ctypes.byref(srv)) == 1
    assert lib.sift_server_create(ctypes.byref(p), ctypes.c_void_p(260), 1 << 30, 8, 2,
                                  ctypes.byref(srv)) == 1
    assert lib.sift_server_create(ctypes.byref(p), ctypes.c_void_p(256), 1 << 30, 0, 2,
                                  ctypes.byref(srv)) == 1
    assert lib.sift_server_create(ctypes.byref(p), ctypes.c_void_p(256), 1 << 30, 8, 9,
                                  ctypes.byref(srv)) == 1
    assert b"max_inflight" in lib.sift_last_error()
    bad = S.make_params(n_scales=0)
    assert lib.sift_server_create(ctypes.byref(bad), ctypes.c_void_p(256), 1 << 30, 8, 2,
                                  ctypes.byref(srv)) == 6
    st = S.SiftServerStats()
    assert lib.sift_server_get_stats(None, ctypes.byref(st)) == 1
    assert lib.sift_server_destroy(None) == 0
    assert ctypes.sizeof(S.SiftServerStats) == 56


def test_graph_and_autotune_argument_errors():
    lib = S.load_library()
    assert lib.sift_graph_launch(None, None) == 1
    assert lib.sift_graph_destroy(None) == 0
    g = ctypes.c_void_p()
    assert lib.sift_graph_create(None, 1, None, None, None, None, None, 0, None, None) == 1
    best = ctypes.c_int32()
    p = S.make_params()
    assert lib.sift_autotune_batch(None, 1, None, None, None, None, None, 0, None, None, 1, 3,
                                   ctypes.byref(best), None) == 1
    assert lib.sift_autotune_batch(ctypes.byref(p), 1, None, None, None, None, None, 0, None,
                                   None, 1, 0, ctypes.byref(best), None) == 1


def test_window_and_scale_limits():
    """Settings whose windows or blur radii the kernels cannot cover are
    refused at create time: s = 1 (an incremental blur of radius 45), a
    descriptor window of 2048 samples or more a side (desc_magnif x largest
    domain size x largest keypoint scale), an orientation window as large."""
    lib = S.load_library()
    h = ctypes.c_void_p()
    for bad in (dict(n_scales=1), dict(dsp_scales=[1.0, 30.0]), dict(desc_magnif=90.0),
                dict(ori_radius_factor=200.0)):
        pp = S.make_params(**bad)
        assert lib.sift_create(ctypes.byref(pp), ctypes.byref(h)) == 6, bad
        assert b"exceeds" in lib.sift_last_error(), bad
    # the largest keypoint scale at s = 3 is 1.6 * 2^(3.5/3) = 3.59 px: a
    # domain size of 26 gives a descriptor half-side ceil(2.5 sqrt 2 * 3 *
    # 3.59 * 26) + 1 = 992, inside the limit; 27 gives 1030, outside
    for ok in (dict(n_scales=2), dict(n_scales=5), dict(n_scales=6), dict(dsp_scales=[26.0])):
        S.Extractor(**ok)
    pp = S.make_params(dsp_scales=[27.5])
    assert lib.sift_create(ctypes.byref(pp), ctypes.byref(h)) == 6

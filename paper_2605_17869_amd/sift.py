"""Python binding of the C ABI in include/sift.h (argument marshalling only).

Every step of extraction runs in the HIP library ``libsift_mi355x.so``; this
module allocates device buffers with torch, passes raw pointers and the
current HIP stream, and converts results.  It refuses to run when the library
is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, fields
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().with_name("libsift_mi355x.so")
# the same library with bounds checks in its kernels (tests)
BOUNDS_LIB_PATH = LIB_PATH.with_name("libsift_mi355x_bounds.so")
MAX_DSP = 16
DESC_DIM = 128

SIFT_OK = 0
STATUS_NAMES = {
    0: "SIFT_OK", 1: "SIFT_ERR_INVALID_ARG", 2: "SIFT_ERR_IMAGE_TOO_SMALL",
    3: "SIFT_ERR_WORKSPACE_TOO_SMALL", 4: "SIFT_ERR_TOO_LARGE", 5: "SIFT_ERR_HIP",
    6: "SIFT_ERR_NOT_SUPPORTED",
}


class SiftParams(ctypes.Structure):
    _fields_ = [
        ("n_octaves", ctypes.c_int32), ("n_scales", ctypes.c_int32), ("upsample", ctypes.c_int32),
        ("sigma0", ctypes.c_float), ("sigma_in", ctypes.c_float),
        ("contrast_threshold", ctypes.c_float), ("prefilter_ratio", ctypes.c_float),
        ("edge_ratio", ctypes.c_float), ("border", ctypes.c_int32),
        ("refine_iters", ctypes.c_int32), ("ori_bins", ctypes.c_int32),
        ("ori_sigma_factor", ctypes.c_float), ("ori_radius_factor", ctypes.c_float),
        ("ori_peak_ratio", ctypes.c_float), ("upright", ctypes.c_int32),
        ("desc_width", ctypes.c_int32), ("desc_ori_bins", ctypes.c_int32),
        ("desc_magnif", ctypes.c_float), ("desc_clamp", ctypes.c_float),
        ("n_dsp", ctypes.c_int32), ("dsp_scales", ctypes.c_float * MAX_DSP),
        ("rootsift", ctypes.c_int32), ("max_keypoints", ctypes.c_int32),
        ("max_candidates", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
        ("n_streams", ctypes.c_int32), ("upsample_max_pixels", ctypes.c_int32),
        ("pyramid_fp16", ctypes.c_int32), ("blur_chain", ctypes.c_int32),
        ("detect_waves", ctypes.c_int32),
    ]


class SiftOutput(ctypes.Structure):
    _fields_ = [
        ("keypoints", ctypes.c_void_p), ("descriptors", ctypes.c_void_p),
        ("count", ctypes.c_void_p), ("n_found", ctypes.c_void_p),
        ("n_candidates", ctypes.c_void_p), ("capacity", ctypes.c_int32),
    ]


class SiftLaunchStat(ctypes.Structure):
    _fields_ = [("stage", ctypes.c_char * 32), ("label", ctypes.c_char * 32),
                ("ms", ctypes.c_double), ("bytes", ctypes.c_double), ("fmas", ctypes.c_double)]


class SiftStageStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int32),
                ("ms", ctypes.c_double), ("bytes", ctypes.c_double)]


KEYPOINT_DTYPE = np.dtype([
    ("x", "<f4"), ("y", "<f4"), ("sigma", "<f4"), ("angle", "<f4"), ("response", "<f4"),
    ("octave", "<i4"), ("layer", "<i4"), ("ix", "<i4"), ("iy", "<i4"),
    ("src_layer", "<i4"), ("src_iy", "<i4"), ("src_ix", "<i4"),
])
assert KEYPOINT_DTYPE.itemsize == 48

class SiftServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("peak_arena", ctypes.c_int64),
                ("peak_inflight", ctypes.c_int64), ("largest_batch", ctypes.c_int64),
                ("overlapped_batches", ctypes.c_int64)]


class SiftMatchPair(ctypes.Structure):
    _fields_ = [("desc_a", ctypes.c_void_p), ("count_a", ctypes.c_void_p), ("cap_a", ctypes.c_int32),
                ("desc_b", ctypes.c_void_p), ("count_b", ctypes.c_void_p), ("cap_b", ctypes.c_int32),
                ("matches", ctypes.c_void_p), ("n_matches", ctypes.c_void_p),
                ("n_found", ctypes.c_void_p), ("capacity", ctypes.c_int32)]


class SiftVerifyPair(ctypes.Structure):
    _fields_ = [("kp_a", ctypes.c_void_p), ("kp_b", ctypes.c_void_p), ("matches", ctypes.c_void_p),
                ("n_matches", ctypes.c_void_p), ("cap", ctypes.c_int32), ("H", ctypes.c_void_p),
                ("score", ctypes.c_void_p), ("n_inliers", ctypes.c_void_p),
                ("best", ctypes.c_void_p), ("weights", ctypes.c_void_p)]


MATCH_DTYPE = np.dtype([("query", "<i4"), ("train", "<i4"), ("similarity", "<f4"),
                        ("distance", "<f4")])


class SiftTuning(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("ms", ctypes.c_float), ("from_cache", ctypes.c_int32), ("n_tried", ctypes.c_int32),
                ("blur_chain", ctypes.c_int32), ("detect_waves", ctypes.c_int32)]


# name -> (restype, argtypes)
_SIGNATURES = {
    "sift_params_default": (ctypes.c_int, [ctypes.POINTER(SiftParams)]),
    "sift_create": (ctypes.c_int, [ctypes.POINTER(SiftParams), ctypes.POINTER(ctypes.c_void_p)]),
    "sift_destroy": (None, [ctypes.c_void_p]),
    "sift_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SiftParams)]),
    "sift_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_size_t)]),
    "sift_extract": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_size_t, ctypes.POINTER(SiftOutput), ctypes.c_void_p]),
    "sift_batch_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                                 ctypes.POINTER(ctypes.c_int32),
                                                 ctypes.POINTER(ctypes.c_int32),
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "sift_extract_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.POINTER(SiftOutput),
                                          ctypes.c_void_p]),
    "sift_workspace_level": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_void_p),
                                            ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32)]),
    "sift_workspace_level_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "sift_profile_start": (ctypes.c_int, []),
    "sift_profile_stop": (ctypes.c_int, [ctypes.POINTER(SiftStageStat), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32)]),
    "sift_profile_launches": (ctypes.c_int, [ctypes.POINTER(SiftLaunchStat), ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_int32)]),
    "sift_server_create": (ctypes.c_int, [ctypes.POINTER(SiftParams), ctypes.c_void_p,
                                          ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "sift_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int64,
                                          ctypes.POINTER(SiftOutput),
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "sift_server_submit_n": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_void_p),
                                            ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int32),
                                            ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(SiftOutput),
                                            ctypes.POINTER(ctypes.c_uint64)]),
    "sift_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_double)]),
    "sift_server_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_double)]),
    "sift_server_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(SiftServerStats)]),
    "sift_server_batch_bytes": (ctypes.c_int, [ctypes.POINTER(SiftParams), ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_int32),
                                               ctypes.POINTER(ctypes.c_int32),
                                               ctypes.POINTER(ctypes.c_size_t)]),
    "sift_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sift_graph_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_void_p),
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p,
                                         ctypes.c_size_t, ctypes.POINTER(SiftOutput),
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "sift_graph_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sift_graph_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sift_autotune_batch": (ctypes.c_int, [ctypes.POINTER(SiftParams), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p,
                                           ctypes.c_size_t, ctypes.POINTER(SiftOutput),
                                           ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_float)]),
    "sift_extract_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_int64,
                                            ctypes.POINTER(SiftOutput), ctypes.c_void_p]),
    "sift_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "sift_match_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(SiftMatchPair),
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "sift_match_batch": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(SiftMatchPair),
                                        ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p]),
    "sift_bucket_workspace_size": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "sift_bucket_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "sift_bucket_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_void_p),
                                          ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(SiftOutput), ctypes.c_void_p]),
    "sift_bucket_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sift_autotune": (ctypes.c_int, [ctypes.POINTER(SiftParams), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_void_p),
                                     ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.POINTER(SiftOutput), ctypes.c_void_p,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_char_p, ctypes.POINTER(SiftTuning)]),
    "sift_autotune_workspace_size": (ctypes.c_int, [ctypes.POINTER(SiftParams), ctypes.c_int32,
                                                    ctypes.POINTER(ctypes.c_int32),
                                                    ctypes.POINTER(ctypes.c_int32),
                                                    ctypes.POINTER(ctypes.c_size_t)]),
    "sift_verify_workspace_size": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(SiftVerifyPair),
                                                  ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "sift_verify_batch": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(SiftVerifyPair),
                                         ctypes.c_void_p, ctypes.c_int32, ctypes.c_float,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t,
                                         ctypes.c_void_p]),
    "sift_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "sift_bounds_violations": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]),
    "sift_last_error": (ctypes.c_char_p, []),
}

_lib = None
_bounds_lib = None


class SiftError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {detail}")
        self.status = status


def _open(path: Path):
    if not path.exists():
        raise ImportError(f"{path} is missing: build it with "
                          f"`python -m paper_2605_17869_amd.build`")
    # torch first: the library then binds to the HIP runtime torch already
    # loaded (same soname), so the process holds a single runtime
    import torch  # noqa: F401
    lib = ctypes.CDLL(str(path))
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def load_library(bounds: bool = False):
    """Load libsift_mi355x.so (built by ``python -m paper_2605_17869_amd.build``),
    or with ``bounds`` its twin whose kernels count out-of-range accesses."""
    global _lib, _bounds_lib
    if bounds:
        if _bounds_lib is None:
            _bounds_lib = _open(BOUNDS_LIB_PATH)
        return _bounds_lib
    if _lib is None:
        _lib = _open(LIB_PATH)
    return _lib


def _check(status: int, where: str):
    if status != SIFT_OK:
        # the message is kept by the library that failed: the loaded ones are asked
        detail = ""
        for lib in (_lib, _bounds_lib):
            if lib is not None and not detail:
                detail = lib.sift_last_error().decode()
        raise SiftError(status, where, detail)


def bounds_violations(reset: bool = True) -> int:
    """``sift_bounds_violations`` of the bounds-checked library: out-of-range
    accesses its kernels counted since the last reset (waits for the device)."""
    n = ctypes.c_uint64()
    _check(load_library(bounds=True).sift_bounds_violations(1 if reset else 0, ctypes.byref(n)),
           "sift_bounds_violations")
    return int(n.value)


def make_params(settings: dict | None = None, **overrides) -> SiftParams:
    """sift_params from the library defaults updated by ``settings`` (a dict
    with sift_params field names; ``dsp_scales`` a sequence)."""
    lib = load_library()
    p = SiftParams()
    _check(lib.sift_params_default(ctypes.byref(p)), "sift_params_default")
    merged = dict(settings or {})
    merged.update(overrides)
    names = {f[0] for f in SiftParams._fields_}
    for key, val in merged.items():
        if key == "dsp_scales":
            vals = [float(v) for v in val]
            if not 1 <= len(vals) <= MAX_DSP:
                raise ValueError("dsp_scales needs 1..16 entries")
            p.n_dsp = len(vals)
            for i in range(MAX_DSP):
                p.dsp_scales[i] = vals[i] if i < len(vals) else 0.0
        elif key in names:
            setattr(p, key, type(getattr(p, key))(val))
    return p


@dataclass
class Features:
    """Device-resident results of one image (torch tensors on the GPU)."""
    keypoints: object      # int32 [capacity, 12]: sift_keypoint records
    descriptors: object    # float32 [capacity, 128]
    counters: object       # int32 [3]: count, n_found, n_candidates

    def host(self):
        """(keypoints as a KEYPOINT_DTYPE array, descriptors, n_found, n_candidates)."""
        cnt = self.counters.cpu().numpy()
        n = int(cnt[0])
        kp = self.keypoints[:n].cpu().numpy().copy().view(KEYPOINT_DTYPE).reshape(-1)
        desc = self.descriptors[:n].cpu().numpy().copy()
        return kp, desc, int(cnt[1]), int(cnt[2])


def profile_start():
    """Begin recording per-stage HIP events for every extraction."""
    _check(load_library().sift_profile_start(), "sift_profile_start")


def profile_stop() -> dict:
    """Wait for recorded stages; {stage: (launches, ms, algorithmic bytes)}."""
    arr = (SiftStageStat * 16)()
    n = ctypes.c_int32()
    _check(load_library().sift_profile_stop(arr, 16, ctypes.byref(n)), "sift_profile_stop")
    return {arr[i].name.decode(): (arr[i].launches, arr[i].ms, arr[i].bytes)
            for i in range(n.value)}


def profile_launches(max_launches: int = 4096) -> list:
    """Recorded launches so far: [(stage, label, ms, bytes, fmas)] in enqueue order."""
    arr = (SiftLaunchStat * max_launches)()
    n = ctypes.c_int32()
    _check(load_library().sift_profile_launches(arr, max_launches, ctypes.byref(n)),
           "sift_profile_launches")
    return [(arr[i].stage.decode(), arr[i].label.decode(), arr[i].ms, arr[i].bytes, arr[i].fmas)
            for i in range(n.value)]


def _stream_handle(stream) -> ctypes.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Extractor:
    """Handle around ``sift_create``; extraction allocates outputs and a
    workspace with torch on the current device and enqueues on the current
    (or given) stream."""

    def __init__(self, settings: dict | None = None, bounds_checked: bool = False, **overrides):
        # bounds_checked: run on the library whose kernels count out-of-range
        # accesses (same results; see bounds_violations)
        self.lib = load_library(bounds=bounds_checked)
        self.params = make_params(settings, **overrides)
        h = ctypes.c_void_p()
        _check(self.lib.sift_create(ctypes.byref(self.params), ctypes.byref(h)), "sift_create")
        self.handle = h
        self._ws = None

    def __del__(self):
        lib, h = getattr(self, "lib", None), getattr(self, "handle", None)
        if lib is not None and h is not None and h.value:
            lib.sift_destroy(h)
            self.handle = None

    def workspace_size(self, height: int, width: int) -> int:
        n = ctypes.c_size_t()
        _check(self.lib.sift_workspace_size(self.handle, height, width, ctypes.byref(n)),
               "sift_workspace_size")
        return n.value

    def batch_workspace_size(self, sizes) -> int:
        n = len(sizes)
        hs = (ctypes.c_int32 * n)(*[int(h) for h, _ in sizes])
        ws = (ctypes.c_int32 * n)(*[int(w) for _, w in sizes])
        out = ctypes.c_size_t()
        _check(self.lib.sift_batch_workspace_size(self.handle, n, hs, ws, ctypes.byref(out)),
               "sift_batch_workspace_size")
        return out.value

    def workspace(self, nbytes: int):
        """A cached device workspace of at least nbytes."""
        import torch
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        return self._ws

    def alloc_features(self, capacity: int | None = None) -> Features:
        import torch
        cap = int(self.params.max_keypoints if capacity is None else capacity)
        return Features(torch.empty((max(cap, 1), 12), dtype=torch.int32, device="cuda"),
                        torch.empty((max(cap, 1), DESC_DIM), dtype=torch.float32, device="cuda"),
                        torch.zeros(3, dtype=torch.int32, device="cuda"))

    @staticmethod
    def _output(f: Features, capacity: int) -> SiftOutput:
        base = f.counters.data_ptr()
        return SiftOutput(f.keypoints.data_ptr(), f.descriptors.data_ptr(), base, base + 4,
                          base + 8, capacity)

    def extract(self, image, capacity: int | None = None, out: Features | None = None,
                workspace=None, stream=None) -> Features:
        """Enqueue extraction of one 2-D float32 CUDA tensor."""
        import torch
        if image.dim() != 2 or image.dtype != torch.float32 or not image.is_cuda:
            raise ValueError("image must be a 2-D float32 CUDA tensor")
        if image.stride(1) != 1:
            raise ValueError("image rows must be contiguous")
        h, w = image.shape
        need = self.workspace_size(h, w)
        ws = workspace if workspace is not None else self.workspace(need)
        f = out if out is not None else self.alloc_features(capacity)
        cap = f.keypoints.shape[0] if capacity is None else int(capacity)
        o = self._output(f, cap)
        _check(self.lib.sift_extract(self.handle, ctypes.c_void_p(image.data_ptr()), h, w,
                                     image.stride(0), ctypes.c_void_p(ws.data_ptr()),
                                     ws.numel() * ws.element_size(), ctypes.byref(o),
                                     _stream_handle(stream)), "sift_extract")
        return f

    def extract_noalloc(self, image, out: Features, capacity: int | None = None,
                        stream=None) -> Features:
        """``sift_extract_noalloc``: extraction into the library's static
        device scratch (no workspace argument, nothing allocated here either:
        ``out`` is the caller's)."""
        import torch
        if image.dim() != 2 or image.dtype != torch.float32 or not image.is_cuda:
            raise ValueError("image must be a 2-D float32 CUDA tensor")
        if image.stride(1) != 1:
            raise ValueError("image rows must be contiguous")
        h, w = image.shape
        cap = out.keypoints.shape[0] if capacity is None else int(capacity)
        o = self._output(out, cap)
        _check(self.lib.sift_extract_noalloc(self.handle, ctypes.c_void_p(image.data_ptr()), h, w,
                                             image.stride(0), ctypes.byref(o),
                                             _stream_handle(stream)), "sift_extract_noalloc")
        return out

    def _batch_args(self, images, capacity, outs, workspace):
        import torch
        n = len(images)
        for im in images:
            if im.dim() != 2 or im.dtype != torch.float32 or not im.is_cuda or im.stride(1) != 1:
                raise ValueError("images must be 2-D CUDA tensors with contiguous rows")
        sizes = [tuple(im.shape) for im in images]
        need = self.batch_workspace_size(sizes)
        ws = workspace if workspace is not None else self.workspace(need)
        feats = outs if outs is not None else [self.alloc_features(capacity) for _ in range(n)]
        ptrs = (ctypes.c_void_p * n)(*[im.data_ptr() for im in images])
        hs = (ctypes.c_int32 * n)(*[s[0] for s in sizes])
        wss = (ctypes.c_int32 * n)(*[s[1] for s in sizes])
        pitches = (ctypes.c_int64 * n)(*[im.stride(0) for im in images])
        o = (SiftOutput * n)(*[self._output(f, f.keypoints.shape[0] if capacity is None
                                            else int(capacity)) for f in feats])
        return (n, ptrs, hs, wss, pitches, ctypes.c_void_p(ws.data_ptr()),
                ws.numel() * ws.element_size(), o), feats, ws

    def extract_batch(self, images, capacity: int | None = None, outs=None, workspace=None,
                      stream=None) -> list:
        """Enqueue extraction of a list of 2-D float32 CUDA tensors in one batch."""
        args, feats, _ = self._batch_args(images, capacity, outs, workspace)
        _check(self.lib.sift_extract_batch(self.handle, *args, _stream_handle(stream)),
               "sift_extract_batch")
        return feats

    def graph(self, images, capacity: int | None = None, outs=None, workspace=None):
        """Record the batch's launch sequence into a replayable graph (the
        images are read at their current addresses on every replay)."""
        import torch
        if workspace is None:   # a graph owns its workspace: replays must not share it
            workspace = torch.empty(self.batch_workspace_size([tuple(im.shape) for im in images]),
                                    dtype=torch.uint8, device="cuda")
        args, feats, ws = self._batch_args(images, capacity, outs, workspace)
        g = ctypes.c_void_p()
        _check(self.lib.sift_graph_create(self.handle, *args, ctypes.byref(g)),
               "sift_graph_create")
        return BatchGraph(self.lib, g, list(images), feats, ws)

    def bucket(self, n_slots: int, max_height: int, max_width: int):
        """A replayable launch sequence for up to n_slots images of at most
        max_height x max_width (``sift_bucket_*``); owns its workspace."""
        import torch
        need = ctypes.c_size_t()
        _check(self.lib.sift_bucket_workspace_size(self.handle, n_slots, max_height, max_width,
                                                   ctypes.byref(need)), "sift_bucket_workspace_size")
        ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
        hb = ctypes.c_void_p()
        _check(self.lib.sift_bucket_create(self.handle, n_slots, max_height, max_width,
                                           ctypes.c_void_p(ws.data_ptr()), need.value,
                                           ctypes.byref(hb)), "sift_bucket_create")
        return Bucket(self, hb, ws, n_slots)

    def autotune(self, images, warmup: int = 1, reps: int = 3, outs=None, workspace=None,
                 stream=None):
        """(best tile_rows, {tile_rows: ms}) for this batch; see sift_autotune_batch."""
        args, _, _ = self._batch_args(images, None, outs, workspace)
        best = ctypes.c_int32()
        ms = (ctypes.c_float * 4)()
        _check(self.lib.sift_autotune_batch(ctypes.byref(self.params), *args,
                                            _stream_handle(stream), warmup, reps,
                                            ctypes.byref(best), ms), "sift_autotune_batch")
        return best.value, dict(zip((64, 128, 256, 512), list(ms)))

    def tune(self, images, warmup: int = 1, reps: int = 3, cache_path: str | None = None,
             as_graph: bool = False, outs=None, workspace=None, stream=None) -> dict:
        """``sift_autotune``: the fastest (tile_rows, n_streams, blur_chain,
        detect_waves) for this batch run as a launch sequence (or, ``as_graph``,
        as graph replays), from ``cache_path`` when it holds the batch's key."""
        import torch
        if workspace is None:
            n = len(images)
            hs = (ctypes.c_int32 * n)(*[int(im.shape[0]) for im in images])
            wss = (ctypes.c_int32 * n)(*[int(im.shape[1]) for im in images])
            need = ctypes.c_size_t()
            _check(self.lib.sift_autotune_workspace_size(ctypes.byref(self.params), n, hs, wss,
                                                         ctypes.byref(need)),
                   "sift_autotune_workspace_size")
            workspace = torch.empty(need.value, dtype=torch.uint8, device="cuda")
        args, _, _ = self._batch_args(images, None, outs, workspace)
        t = SiftTuning()
        path = cache_path.encode() if cache_path else None
        _check(self.lib.sift_autotune(ctypes.byref(self.params), *args, _stream_handle(stream),
                                      warmup, reps, 1 if as_graph else 0, path, ctypes.byref(t)),
               "sift_autotune")
        return {"tile_rows": t.tile_rows, "n_streams": t.n_streams, "blur_chain": t.blur_chain,
                "detect_waves": t.detect_waves, "ms": round(t.ms, 4),
                "from_cache": bool(t.from_cache), "candidates_timed": t.n_tried,
                "timed_as": "graph replay" if as_graph else "launch sequence"}

    def level(self, workspace, height: int, width: int, octave: int, level: int):
        """Gaussian level (octave, level) of the last single-image extraction in
        ``workspace`` as a float32 numpy array (L, not L - 0.5)."""
        import torch
        ptr = ctypes.c_void_p()
        lh, lw, lp = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.sift_workspace_level(self.handle, height, width,
                                             ctypes.c_void_p(workspace.data_ptr()), octave, level,
                                             ctypes.byref(ptr), ctypes.byref(lh),
                                             ctypes.byref(lw), ctypes.byref(lp)),
               "sift_workspace_level")
        es = ctypes.c_int32()
        _check(self.lib.sift_workspace_level_bytes(self.handle, height, width, octave,
                                                   ctypes.byref(es)), "sift_workspace_level_bytes")
        off = ptr.value - workspace.data_ptr()
        n = lh.value * lp.value
        dt = torch.float16 if es.value == 2 else torch.float32
        flat = workspace[off:off + es.value * n].view(dt)
        arr = flat.view(lh.value, lp.value)[:, :lw.value].float().cpu().numpy().astype(np.float64)
        return arr + 0.5


class Bucket:
    """A size bucket (``sift_bucket_*``): replays its recorded launch sequence
    for any images that fit; keeps its extractor and workspace alive."""

    def __init__(self, extractor, handle, workspace, n_slots):
        self.ex, self.handle, self._ws, self.n_slots = extractor, handle, workspace, n_slots

    def launch(self, images, outs=None, capacity: int | None = None, stream=None) -> list:
        import torch
        n = len(images)
        for im in images:
            if im.dim() != 2 or im.dtype != torch.float32 or not im.is_cuda or im.stride(1) != 1:
                raise ValueError("images must be 2-D CUDA tensors with contiguous rows")
        feats = outs if outs is not None else [self.ex.alloc_features(capacity) for _ in range(n)]
        ptrs = (ctypes.c_void_p * n)(*[im.data_ptr() for im in images])
        hs = (ctypes.c_int32 * n)(*[im.shape[0] for im in images])
        wss = (ctypes.c_int32 * n)(*[im.shape[1] for im in images])
        pitches = (ctypes.c_int64 * n)(*[im.stride(0) for im in images])
        o = (SiftOutput * n)(*[self.ex._output(f, f.keypoints.shape[0] if capacity is None
                                               else int(capacity)) for f in feats])
        _check(self.ex.lib.sift_bucket_launch(self.handle, n, ptrs, hs, wss, pitches, o,
                                              _stream_handle(stream)), "sift_bucket_launch")
        return feats

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            st = self.ex.lib.sift_bucket_destroy(self.handle)
            self.handle = None
            _check(st, "sift_bucket_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchGraph:
    """A recorded batch (``sift_graph_*``); keeps its buffers alive."""

    def __init__(self, lib, handle, images, feats, workspace):
        self.lib, self.handle = lib, handle
        self.images, self.features, self._ws = images, feats, workspace

    def launch(self, stream=None):
        _check(self.lib.sift_graph_launch(self.handle, _stream_handle(stream)),
               "sift_graph_launch")
        return self.features

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            st = self.lib.sift_graph_destroy(self.handle)
            self.handle = None
            _check(st, "sift_graph_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def server_batch_bytes(settings: dict | None, sizes) -> int:
    """Arena bytes a server reserves for one batch of images of ``sizes``
    ((height, width) pairs): ``sift_server_batch_bytes``."""
    lib = load_library()
    p = make_params(settings)
    n = len(sizes)
    hs = (ctypes.c_int32 * n)(*[int(h) for h, _ in sizes])
    ws = (ctypes.c_int32 * n)(*[int(w) for _, w in sizes])
    out = ctypes.c_size_t()
    _check(lib.sift_server_batch_bytes(ctypes.byref(p), n, hs, ws, ctypes.byref(out)),
           "sift_server_batch_bytes")
    return out.value


class Server:
    """Continuous-batching server (``sift_server_*``) over a torch-allocated
    device arena.  ``submit`` returns a ticket at once; ``wait`` / ``poll``
    report completion and the request's latency in milliseconds."""

    def __init__(self, settings: dict | None = None, arena_bytes: int = 1 << 32,
                 max_batch: int = 64, max_inflight: int = 2, **overrides):
        import torch
        self.lib = load_library()
        self.params = make_params(settings, **overrides)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()   # the arena exists before the worker uses it
        h = ctypes.c_void_p()
        _check(self.lib.sift_server_create(ctypes.byref(self.params),
                                           ctypes.c_void_p(self.arena.data_ptr()),
                                           int(arena_bytes), int(max_batch), int(max_inflight),
                                           ctypes.byref(h)), "sift_server_create")
        self.handle = h
        self._held = {}   # ticket -> (image, features) kept alive until reported

    def alloc_features(self, capacity: int | None = None) -> Features:
        import torch
        cap = int(self.params.max_keypoints if capacity is None else capacity)
        return Features(torch.empty((max(cap, 1), 12), dtype=torch.int32, device="cuda"),
                        torch.empty((max(cap, 1), DESC_DIM), dtype=torch.float32, device="cuda"),
                        torch.zeros(3, dtype=torch.int32, device="cuda"))

    def submit(self, image, out: Features | None = None) -> int:
        """Enqueue one 2-D float32 CUDA tensor (already written: the caller
        synchronises its own stream first); returns the ticket."""
        import torch
        if image.dim() != 2 or image.dtype != torch.float32 or not image.is_cuda or \
                image.stride(1) != 1:
            raise ValueError("image must be a 2-D float32 CUDA tensor with contiguous rows")
        f = out if out is not None else self.alloc_features()
        o = Extractor._output(f, f.keypoints.shape[0])
        t = ctypes.c_uint64()
        h, w = image.shape
        _check(self.lib.sift_server_submit(self.handle, ctypes.c_void_p(image.data_ptr()), h, w,
                                           image.stride(0), ctypes.byref(o), ctypes.byref(t)),
               "sift_server_submit")
        self._held[t.value] = (image, f)
        return t.value

    def submit_many(self, images, outs=None) -> list:
        """Enqueue several 2-D float32 CUDA tensors as one group (they join
        the queue together); returns their tickets."""
        import torch
        n = len(images)
        for im in images:
            if im.dim() != 2 or im.dtype != torch.float32 or not im.is_cuda or im.stride(1) != 1:
                raise ValueError("images must be 2-D float32 CUDA tensors with contiguous rows")
        feats = list(outs) if outs is not None else [self.alloc_features() for _ in range(n)]
        ptrs = (ctypes.c_void_p * n)(*[im.data_ptr() for im in images])
        hs = (ctypes.c_int32 * n)(*[im.shape[0] for im in images])
        ws = (ctypes.c_int32 * n)(*[im.shape[1] for im in images])
        ps = (ctypes.c_int64 * n)(*[im.stride(0) for im in images])
        os_ = (SiftOutput * n)(*[Extractor._output(f, f.keypoints.shape[0]) for f in feats])
        ts = (ctypes.c_uint64 * n)()
        _check(self.lib.sift_server_submit_n(self.handle, n, ptrs, hs, ws, ps, os_, ts),
               "sift_server_submit_n")
        for k in range(n):
            self._held[ts[k]] = (images[k], feats[k])
        return list(ts)

    def poll(self, ticket: int):
        """(done, latency_ms, features) -- latency and features once done."""
        done = ctypes.c_int32()
        lat = ctypes.c_double()
        _check(self.lib.sift_server_poll(self.handle, ticket, ctypes.byref(done),
                                         ctypes.byref(lat)), "sift_server_poll")
        if not done.value:
            return False, None, None
        return True, lat.value, self._held.pop(ticket)[1]

    def wait(self, ticket: int):
        """Block until done; returns (latency_ms, features)."""
        lat = ctypes.c_double()
        _check(self.lib.sift_server_wait(self.handle, ticket, ctypes.byref(lat)),
               "sift_server_wait")
        return lat.value, self._held.pop(ticket)[1]

    def stats(self) -> dict:
        st = SiftServerStats()
        _check(self.lib.sift_server_get_stats(self.handle, ctypes.byref(st)),
               "sift_server_get_stats")
        return {k: getattr(st, k) for k, _ in SiftServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            st = self.lib.sift_server_destroy(self.handle)
            self.handle = None
            self._held.clear()
            _check(st, "sift_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Matches:
    """Device-resident matches of one pair (torch tensors on the GPU)."""
    records: object        # int32 [capacity, 4]: sift_match records
    counters: object       # int32 [2]: n_matches, n_found

    def host(self):
        """(matches as a MATCH_DTYPE array, n_found)."""
        cnt = self.counters.cpu().numpy()
        n = int(cnt[0])
        rec = self.records[:n].cpu().numpy().copy().view(MATCH_DTYPE).reshape(-1)
        return rec, int(cnt[1])


def _desc_arg(desc, count):
    import torch
    if desc.dim() != 2 or desc.shape[1] != DESC_DIM or desc.dtype != torch.float32 \
            or not desc.is_cuda or not desc.is_contiguous():
        raise ValueError("descriptors must be a contiguous float32 CUDA tensor [rows, 128]")
    cptr = None
    if count is not None:
        if count.dtype != torch.int32 or not count.is_cuda:
            raise ValueError("count must be an int32 CUDA tensor")
        cptr = count.data_ptr()
    return desc.data_ptr() if desc.shape[0] else None, cptr, int(desc.shape[0])


def match_batch(pairs, ratio: float = 0.8, workspace=None, stream=None, outs=None,
                bounds_checked: bool = False) -> list:
    """``sift_match_batch`` over pairs of (desc_a, count_a, desc_b, count_b):
    descriptors are float32 CUDA tensors [cap, 128]; a count is a one-element
    int32 CUDA tensor holding the rows in use (e.g. ``Features.counters[0:1]``)
    or None for all rows.  Returns one ``Matches`` per pair (enqueued on the
    current or given stream); ``outs`` reuses the ``Matches`` of an earlier call
    on pairs of the same sizes; ``bounds_checked`` runs the bounds-checked library."""
    import torch
    lib = load_library(bounds=bounds_checked)
    n = len(pairs)
    arr = (SiftMatchPair * n)()
    reuse = outs is not None
    outs = list(outs) if reuse else []
    for i, (da, ca, db, cb) in enumerate(pairs):
        pa, qa, na = _desc_arg(da, ca)
        pb, qb, nb = _desc_arg(db, cb)
        if reuse:
            m = outs[i]
            cap = int(m.records.shape[0])
        else:
            cap = max(min(na, nb), 1)
            m = Matches(torch.empty((cap, 4), dtype=torch.int32, device="cuda"),
                        torch.zeros(2, dtype=torch.int32, device="cuda"))
            outs.append(m)
        base = m.counters.data_ptr()
        arr[i] = SiftMatchPair(pa, qa, na, pb, qb, nb, m.records.data_ptr(), base, base + 4, cap)
    need = ctypes.c_size_t()
    _check(lib.sift_match_workspace_size(n, arr, ctypes.byref(need)), "sift_match_workspace_size")
    ws = workspace
    if ws is None or ws.numel() * ws.element_size() < need.value:
        ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device="cuda")
    _check(lib.sift_match_batch(n, arr, ctypes.c_float(ratio), ctypes.c_void_p(ws.data_ptr()),
                                ws.numel() * ws.element_size(), _stream_handle(stream)),
           "sift_match_batch")
    for m in outs:
        m._ws = ws   # keep the workspace alive with the results
    return outs


def match(desc_a, desc_b, ratio: float = 0.8, count_a=None, count_b=None, stream=None) -> Matches:
    """One pair: see ``match_batch``."""
    return match_batch([(desc_a, count_a, desc_b, count_b)], ratio=ratio, stream=stream)[0]


@dataclass
class Verification:
    """Device-resident result of verifying one pair (torch tensors on the GPU)."""
    H: object              # float64 [9], row-major, h33 = 1 (NaN: no hypothesis)
    score: object          # float64 [1]
    ints: object           # int32 [2]: n_inliers, best hypothesis (-1: none)
    weights: object        # float32 [cap]: final weight per correspondence

    def host(self):
        """(H as a 3 x 3 numpy array, score, n_inliers, best, weights)."""
        i = self.ints.cpu().numpy()
        return (self.H.cpu().numpy().reshape(3, 3), float(self.score.cpu().item()), int(i[0]),
                int(i[1]), self.weights.cpu().numpy())


def verify_batch(pairs, samples, sigma_max: float = 2.0, refine_iters: int = 5, workspace=None,
                 stream=None, outs=None, bounds_checked: bool = False) -> list:
    """``sift_verify_batch`` over pairs of (kp_a, kp_b, matches, n_matches):
    keypoint tensors as ``Features.keypoints`` (int32 [cap, 12]), matches as
    ``Matches.records`` (int32 [cap, 4]) and n_matches a one-element int32
    tensor (e.g. ``Matches.counters[0:1]``) or None for every row; ``samples``
    a float32 CUDA tensor [n_hyp, 4] of numbers in [0, 1); ``bounds_checked`` runs the
    bounds-checked library."""
    import torch
    lib = load_library(bounds=bounds_checked)
    if samples.dim() != 2 or samples.shape[1] != 4 or samples.dtype != torch.float32 \
            or not samples.is_cuda or not samples.is_contiguous():
        raise ValueError("samples must be a contiguous float32 CUDA tensor [n_hyp, 4]")
    n = len(pairs)
    arr = (SiftVerifyPair * n)()
    res = list(outs) if outs is not None else []
    for i, (ka, kb, m, cnt) in enumerate(pairs):
        cap = int(m.shape[0])
        if outs is None:
            res.append(Verification(torch.empty(9, dtype=torch.float64, device="cuda"),
                                    torch.empty(1, dtype=torch.float64, device="cuda"),
                                    torch.empty(2, dtype=torch.int32, device="cuda"),
                                    torch.empty(max(cap, 1), dtype=torch.float32, device="cuda")))
        v = res[i]
        ib = v.ints.data_ptr()
        arr[i] = SiftVerifyPair(ka.data_ptr(), kb.data_ptr(), m.data_ptr(),
                                cnt.data_ptr() if cnt is not None else None, cap,
                                v.H.data_ptr(), v.score.data_ptr(), ib, ib + 4,
                                v.weights.data_ptr())
    need = ctypes.c_size_t()
    _check(lib.sift_verify_workspace_size(n, arr, int(samples.shape[0]), ctypes.byref(need)),
           "sift_verify_workspace_size")
    ws = workspace
    if ws is None or ws.numel() * ws.element_size() < need.value:
        ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device="cuda")
    _check(lib.sift_verify_batch(n, arr, ctypes.c_void_p(samples.data_ptr()), int(samples.shape[0]),
                                 ctypes.c_float(sigma_max), refine_iters,
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                 _stream_handle(stream)), "sift_verify_batch")
    for v in res:
        v._ws = ws
    return res

"""Helpers shared by the GPU tests: run the HIP path on numpy images."""
from __future__ import annotations

import hashlib
import sys

import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return torch


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def extract(ex, img: np.ndarray, capacity: int | None = None, keep_ws: bool = False):
    """Run sift_extract on one image; returns (kps, desc, n_found, n_cand[, ws])."""
    torch = require_gpu()
    t = torch.from_numpy(np.ascontiguousarray(img, dtype=np.float32)).cuda()
    ws = torch.empty(ex.workspace_size(*img.shape), dtype=torch.uint8, device="cuda")
    f = ex.extract(t, capacity=capacity, workspace=ws)
    torch.cuda.synchronize()
    kp, desc, nf, nc = f.host()
    if keep_ws:
        return kp, desc, nf, nc, ws
    return kp, desc, nf, nc


def extract_batch(ex, imgs, capacity: int | None = None):
    torch = require_gpu()
    ts = [torch.from_numpy(np.ascontiguousarray(i, dtype=np.float32)).cuda() for i in imgs]
    feats = ex.extract_batch(ts, capacity=capacity)
    torch.cuda.synchronize()
    return [f.host() for f in feats]


def digest(kp: np.ndarray, desc: np.ndarray) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(kp).tobytes())
    h.update(np.ascontiguousarray(desc).tobytes())
    return h.hexdigest()

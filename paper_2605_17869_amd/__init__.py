"""GPU-resident, deterministic SIFT extraction for MI355X (gfx950).

The extraction path is the HIP library ``libsift_mi355x.so`` behind the C ABI
of ``include/sift.h``; :mod:`.sift` is its Python binding.
"""
from .sift import (DESC_DIM, KEYPOINT_DTYPE, MATCH_DTYPE, Extractor, Features, Matches,  # noqa: F401
                   Server, SiftError, bounds_violations, load_library, make_params, match,
                   match_batch,
                   profile_launches, profile_start, profile_stop,
                   verify_batch)

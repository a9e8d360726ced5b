"""FP64 CPU oracle of the SIFT extraction path (test infrastructure only)."""
from .sift_oracle import *  # noqa: F401,F403
from .sift_oracle import Params, sift, scale_space  # noqa: F401

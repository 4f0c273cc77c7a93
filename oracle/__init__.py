"""FP64 CPU oracle (test infrastructure only; see dpx_oracle's header)."""
from .dpx_oracle import *  # noqa: F401,F403

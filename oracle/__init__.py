"""FP64 CPU reference oracle (test infrastructure only; see sinkhorn_oracle)."""
from .sinkhorn_oracle import *  # noqa: F401,F403
from . import brute  # noqa: F401

"""FP64 CPU oracle (test infrastructure only; see cp_oracle)."""
from .cp_oracle import *  # noqa: F401,F403

"""FP64 CPU oracle (test infrastructure only; see dwd_oracle)."""
from . import dwd_oracle  # noqa: F401

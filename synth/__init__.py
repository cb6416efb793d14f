"""Seeded synthetic inputs (data only; none of the solver's arithmetic)."""
from .generators import *  # noqa: F401,F403
from .generators import (TwoClassSpec, Workload, two_class, SMALL_F64, HDLSS_F32,  # noqa: F401
                         LARGE_BF16, SWEEP_DATA, sweep_grid, request_stream, Request)

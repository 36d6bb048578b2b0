"""FP64 CPU oracle for DIST's differentiable sphere tracing.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py.  The product library never imports it.
"""
from .dist_oracle import *  # noqa: F401,F403

"""FP64 CPU oracle for PbP-QLP -- test infrastructure only.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this package.  It shares no code with the GPU library.
"""
from .pbpqlp_oracle import *  # noqa: F401,F403
from . import qk_mlp_oracle as qk  # noqa: F401

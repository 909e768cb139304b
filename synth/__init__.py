"""Seeded synthetic inputs shared by the oracle, the tests and the bench.

This package holds only input generation (planted-spectrum matrices and their
seeds).  It contains none of the factorization's arithmetic, so the oracle and
the GPU path can both consume its matrices without sharing method code.
"""
from .matrices import *  # noqa: F401,F403
from .learned import *  # noqa: F401,F403

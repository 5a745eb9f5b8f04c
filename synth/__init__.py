"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This package draws inputs only: sets, sparse tf-idf vectors, dense mixtures,
candidate pairs and lists, and the random coefficients a hash family needs.
It holds none of the verification arithmetic (no posterior, no match
counting, no decision rule), so that the GPU path and the oracle can both
consume its output without sharing any of the method's code.
"""
from .generators import *  # noqa: F401,F403

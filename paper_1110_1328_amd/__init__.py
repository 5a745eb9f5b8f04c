"""BayesLSH candidate verification on AMD Instinct MI355X (gfx950).

The compute lives in libbayeslsh.so (hand-written HIP kernels behind the C ABI
of include/bayeslsh.h); this package only marshals torch device tensors into
that ABI.  Importing it does not load the library; the first call does, and
fails loudly if the library has not been built.
"""
from .api import *  # noqa: F401,F403
from .api import (BayesLSHError, Candidates, Context, Result, Signatures, Vectors, all_pairs,  # noqa: F401
                  csr_vectors, decode, dense_vectors, make_result, pairs, query_lists, set_vectors)

__version__ = "0.1.0"

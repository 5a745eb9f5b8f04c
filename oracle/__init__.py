"""CPU oracle for BayesLSH candidate verification -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, deliberately unoptimised restatement of the
paper's method (Satuluri & Parthasarathy, "Bayesian Locality Sensitive
Hashing for Fast Similarity Search"), used to check the GPU library.  Only
the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import it.  The product path never calls it and shares no code with it.

Modules
  posterior  -- posterior quantities of Section 4 (prune probability,
                MAP estimate, concentration probability) for the Jaccard
                (Section 4.1) and cosine (Section 4.2) instantiations, in FP64.
  hashes     -- the two LSH families of Section 4: minhash and sign random
                projections (with the Philox4x32-10 counter generator for
                on-the-fly Gaussian planes).
  reference  -- Algorithm 1 (BayesLSH) and Algorithm 2 (BayesLSH-Lite), the
                exhaustive and maximum-likelihood comparators and exact
                similarity; small cases run in pure Python, large ones in the
                plain C loop of ``ref.c``.

Parity status of each function is listed in its docstring; every function
here is pinned by a ``-m "not gpu"`` test against closed forms, exact
rational arithmetic, high-precision quadrature or brute force, except where
a docstring says "parity unpinned".
"""

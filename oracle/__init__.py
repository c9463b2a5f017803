"""Plain FP64 CPU oracle for the hybrid DH^2 compression of the Helmholtz
single-layer Galerkin matrix (Boerm & Boerst, arXiv 1809.04384).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute this package; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library
and is written to be checked by eye against the paper: every function cites
the section / equation it follows.  Heavy pointwise sums (Galerkin quadrature
of near-field entries) sit in a small plain-C helper, oracle/csrc/quad.c;
everything else is numpy, with numpy.linalg QR / SVD as library steps.

Parity is pinned by tests/test_oracle_*.py against closed forms, exactness
degrees, invariants, brute force on tiny inputs and the paper's own storage
columns (Tables 1 and 3).
"""

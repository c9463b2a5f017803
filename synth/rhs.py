"""Right-hand sides: i.i.d. complex Gaussian columns N(0,1) + i N(0,1)."""
import numpy as np


def complex_gaussian(n, nrhs, seed=0, dtype=np.complex128):
    """Return an (nrhs, n) array; row j is right-hand side j.

    The real parts of all columns are drawn first, then the imaginary parts,
    from numpy's default_rng(seed).  complex64 is obtained by rounding the
    complex128 draw, so both precisions see the same vectors.
    """
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((nrhs, n))
    im = rng.standard_normal((nrhs, n))
    X = re + 1j * im
    return np.ascontiguousarray(X.astype(dtype))

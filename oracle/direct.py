"""Exact sparse direct solves (oracle; test infrastructure).

The paper solves the subdomain problems and the coarse problem exactly, by a sparse direct
method (section 2.4: UMFPACK).  The oracle uses SciPy's SuperLU by default.  For the
subdomains of the 3M-DOF-class laminates it can use LAPACK's banded Cholesky instead
(pbtrf / pbtrs through scipy.linalg), in the matrix's own order: the laminate DOF
numbering (through-thickness planes outermost) makes every subdomain matrix banded, and a
band factor of such a matrix needs several times less memory than SuperLU's fill there.
Both are the same exact solve of an SPD system, up to rounding.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


def band_lower(A):
    """LAPACK lower band storage ab[i - j, j] = A[i, j] of a sparse symmetric matrix."""
    C = A.tocoo()
    m = C.row >= C.col
    r, c, v = C.row[m], C.col[m], C.data[m]
    bw = int((r - c).max()) if r.size else 0
    ab = np.zeros((bw + 1, A.shape[0]))
    ab[r - c, c] = v
    return ab


def factorized(A, method="superlu"):
    """A solve function b -> A^-1 b (b a vector or an n x k block) for SPD A."""
    if method == "superlu":
        lu = spla.splu(A.tocsc())
        return lu.solve
    if method == "band":
        cb = sla.cholesky_banded(band_lower(A), lower=True, overwrite_ab=True,
                                 check_finite=False)
        return lambda b: sla.cho_solve_banded((cb, True), b, check_finite=False)
    raise ValueError(f"unknown direct method {method!r}")

"""Pin of the oracle's direct solves (section 2.4: exact local solves): SuperLU and the
LAPACK band Cholesky in band storage both reproduce a dense solve of the same SPD matrix,
and the band storage holds exactly the lower triangle."""
import numpy as np
import pytest

import workloads
from oracle import direct, fem


@pytest.mark.parametrize("method", ["superlu", "band"])
def test_direct_solves_match_dense(method):
    prob = fem.Problem(workloads.small_flat(nx=3, ny=2))
    K = prob.K
    rng = np.random.default_rng(4)
    b = rng.standard_normal((K.shape[0], 3))
    x = direct.factorized(K, method)(b)
    xd = np.linalg.solve(K.toarray(), b)
    assert np.abs(x - xd).max() <= 1e-9 * np.abs(xd).max()


def test_band_storage_layout():
    prob = fem.Problem(workloads.small_flat(nx=2, ny=2))
    A = prob.K.toarray()
    ab = direct.band_lower(prob.K)
    bw = ab.shape[0] - 1
    n = A.shape[0]
    for d in range(bw + 1):
        assert np.array_equal(ab[d, : n - d], np.diag(A, -d))
    assert np.abs(np.tril(A, -bw - 1)).max() == 0.0

"""The block-CSR product on every row length: a seeded synthetic matrix (gx_matrix_load)
whose rows hold 0 to 95 blocks, so that every straight-line pass count (1 to 11, 7 blocks a
pass), the rounds of 12 passes and a row longer than one round (84 blocks) all run, against
SciPy's product: every entry within 1e-14 of its row's sum of |a| |x|."""
import numpy as np
import pytest
import scipy.sparse as sp

pytestmark = pytest.mark.gpu


def test_spmv_every_row_length():
    import torch
    import paper_1707_04228_amd as gx
    rng = np.random.default_rng(17)
    n_rows = 2000
    lengths = np.tile(np.arange(96), n_rows // 96 + 1)[:n_rows]
    rng.shuffle(lengths)
    rp = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int32)
    col = np.concatenate([np.sort(rng.choice(n_rows, size=k, replace=False)) for k in lengths])
    col = col.astype(np.int32)
    val = rng.standard_normal(9 * len(col))
    s = gx.Solver()
    s.load_matrix(torch.tensor(rp, device="cuda"), torch.tensor(col, device="cuda"),
                  torch.tensor(val, device="cuda"))
    A = sp.bsr_matrix((val.reshape(-1, 3, 3), col, rp), shape=(3 * n_rows, 3 * n_rows)).tocsr()
    for k in range(2):
        x = rng.standard_normal(3 * n_rows)
        y = s.spmv(torch.tensor(x, device="cuda")).cpu().numpy()
        ref = A @ x
        scale = abs(A) @ np.abs(x)
        assert np.all(np.abs(y - ref) <= 1e-14 * scale + 1e-300), k
    assert np.all(y.reshape(-1, 3)[lengths == 0] == 0.0)
    with pytest.raises(gx.GxError):
        s.geneo_setup(torch.zeros(1, dtype=torch.int32, device="cuda"), 1)
    s.close()

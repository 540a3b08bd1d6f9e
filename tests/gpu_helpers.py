"""Shared helpers for the GPU parity tests (conversion of device results for comparison)."""
import numpy as np
import scipy.sparse as sp


def bcsr_to_scipy(rp, col, val, n_nodes):
    rp = rp.cpu().numpy().astype(np.int64)
    col = col.cpu().numpy().astype(np.int64)
    val = val.cpu().numpy().reshape(-1, 3, 3)
    return sp.bsr_matrix((val, col, rp), shape=(3 * n_nodes, 3 * n_nodes)).tocsr()


def oracle_K_with_identity(prob):
    """Oracle K on all DOFs with clamped rows/columns replaced by identity."""
    Kc = prob.K_all.tocsr().copy()
    D = sp.diags(prob.free.astype(float))
    Kc = (D @ Kc @ D + sp.diags((~prob.free).astype(float))).tocsr()
    return Kc


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

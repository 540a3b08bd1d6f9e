"""GenEO coarse space (oracle; test infrastructure).

Section 2.3: in every subdomain a few of the lowest-energy modes of a local generalised
eigenproblem are computed (rigid-body modes and composite low-energy modes, Fig. fig-eig),
multiplied by the partition of unity and combined into a coarse space; the coarse problem
is solved directly.  The paper defers the exact eigenproblem to Spillane et al. (its
reference for GenEO); the reading used here is that form:

    A_j^N p = lambda B_j p,   B_j = Xt_j A_j^o Xt_j,

with A_j^N the stiffness assembled over the elements of Omega_j on the free DOFs of its
nodes (Neumann matrix), A_j^o the same over the elements of Omega_j that also lie in another
subdomain, and Xt_j the partition of unity extended by zero off I_j.  Selected are the
pairs with lambda < tau (at most nev_max), or the nev smallest when nev > 0.  The coarse
basis vectors are z = R_j^T (Xt_j p)|_{I_j}, and K_0 = Z^T K Z is Cholesky-factored.

Solver: ARPACK in shift-invert mode about -sigma (sigma = 1e-3 tau, or 1e-4 when nev is
given), i.e. the largest mu of B p = mu (A^N + sigma B) p; A^N + sigma B is SPD because no
rigid-body mode lies in the null space of B.  B itself is only semi-definite, and ARPACK
(which uses B as its inner product here) can return vectors carrying null(B) components:
for some start vectors such pairs had residuals of the order of ||A^N p||.  The returned
block is therefore purified by one application of (A^N + sigma B)^-1 B, which removes those
components, and a Rayleigh-Ritz step on the pencil (B, A^N + sigma B) over it gives the
pairs.  ARPACK starts from a fixed vector (results do not depend on earlier calls), and
every pair must have a residual below 1e-11 ||A^N||_1 ||p||, else the oracle raises.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .direct import factorized
from .fem import assemble


def local_matrices(dec, j):
    prob = dec.prob
    mesh = prob.mesh
    free = prob.free_idx
    AN = assemble(mesh, prob.Ke, dec.elems[j])[free][:, free]
    Ao = assemble(mesh, prob.Ke, dec.overlap_elems[j])[free][:, free]
    Dj = dec.D[j]
    AN = AN[Dj][:, Dj].tocsc()
    Ao = Ao[Dj][:, Dj].tocsc()
    xt = np.zeros(len(Dj))
    pos = np.searchsorted(Dj, dec.I[j])
    xt[pos] = dec.X[j]
    B = (sp.diags(xt) @ Ao @ sp.diags(xt)).tocsc()
    return AN, B, xt, pos


def solve_local_eigen(AN, B, nev=0, tau=0.1, nev_max=32, tol=1e-13, dense=None,
                      factor="superlu"):
    """Smallest eigenpairs of A^N p = lambda B p by shift-invert (or dense for tiny sizes).

    dense=None picks the dense solver below 600 DOFs, True/False force one or the other.
    factor: the direct method of the shifted matrix A^N + sigma B (see direct.py); ARPACK
    and the purification step share that one factorisation.
    """
    n = AN.shape[0]
    shift = 1e-4 * (tau if tau else 1.0) if nev > 0 else 1e-3 * tau
    if dense or (dense is None and n <= 600):
        M = (AN + shift * B).toarray()
        mu, V = sla.eigh(B.toarray(), M)
        with np.errstate(divide="ignore"):
            lam = 1.0 / mu[::-1] - shift
        V = V[:, ::-1]
        ok = mu[::-1] > 0
        lam, V = lam[ok], V[:, ok]
        k = nev if nev > 0 else min(nev_max, int(np.sum(lam < tau)))
        return lam[:k], V[:, :k]
    k = nev if nev > 0 else min(8, nev_max)
    v0 = np.random.default_rng(n).standard_normal(n)
    Msh = (AN + shift * B).tocsc()
    solve = factorized(Msh, factor)
    opinv = spla.LinearOperator((n, n), matvec=solve, dtype=np.float64)
    while True:
        kk = min(k, n - 2)
        _, V = spla.eigsh(AN, k=kk, M=B, sigma=-shift, which="LM", tol=tol, v0=v0,
                          ncv=min(n - 1, max(2 * kk + 1, kk + 40)), OPinv=opinv)
        V = solve(B @ V)
        mu, C = sla.eigh(V.T @ (B @ V), V.T @ (Msh @ V))
        V = V @ C
        lam = 1.0 / mu - shift
        res = np.linalg.norm(AN @ V - (B @ V) * lam, axis=0) / (
            abs(AN).sum(axis=0).max() * np.linalg.norm(V, axis=0))
        if not np.all(res <= 1e-11):
            raise RuntimeError(f"ARPACK returned an unconverged pair (backward error "
                               f"{res.max():.1e})")
        order = np.argsort(lam)
        lam, V = lam[order], V[:, order]
        if nev > 0:
            return lam[:nev], V[:, :nev]
        if lam[-1] >= tau or k >= nev_max:
            sel = lam < tau
            return lam[sel][:nev_max], V[:, sel][:, :nev_max]
        k = min(2 * k, nev_max)


class Coarse:
    def __init__(self, dec, nev=0, tau=0.1, nev_max=32, dense=None, factor="superlu",
                 progress=None):
        self.dec = dec
        n = dec.prob.n
        cols, self.lams, self.nev = [], [], []
        for j in range(dec.n_sub):
            AN, B, xt, pos = local_matrices(dec, j)
            lam, V = solve_local_eigen(AN, B, nev=nev, tau=tau, nev_max=nev_max, dense=dense,
                                       factor=factor)
            if progress:
                progress(f"eigensolve {j + 1}/{dec.n_sub}: {len(lam)} modes")
            self.lams.append(lam)
            self.nev.append(len(lam))
            for c in range(V.shape[1]):
                z = np.zeros(n)
                z[dec.I[j]] = (xt * V[:, c])[pos]
                cols.append(z)
        self.n0 = len(cols)
        self.Z = np.array(cols).T if cols else np.zeros((n, 0))
        K = dec.prob.K
        self.K0 = self.Z.T @ (K @ self.Z)
        self.K0 = 0.5 * (self.K0 + self.K0.T)
        self.chol = sla.cho_factor(self.K0, lower=True) if self.n0 else None

    def apply(self, r):
        if not self.n0:
            return np.zeros_like(r)
        return self.Z @ sla.cho_solve(self.chol, self.Z.T @ r)

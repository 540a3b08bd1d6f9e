"""Two-level additive Schwarz preconditioner and preconditioned CG (oracle).

Section 2.3, Eq. (eq-pre): CG is applied to P K u = P f with P a two-level overlapping
Schwarz preconditioner.  Local problems are solved exactly by a direct method (the paper
uses UMFPACK, section 2.4; here SuperLU on the same matrices, the same exact solve) and
the coarse problem directly.  Reading (additive two-level form):

    P r = Z K_0^{-1} Z^T r + sum_j R_j^T A_j^{-1} R_j r,   A_j = K[I_j, I_j],

dropping the first term gives the one-level method of section 2.4.

CG (section 2.3): x_0 = 0 unless given, stop when ||r||_2 <= rtol ||b||_2 (true residual
recurrence, unpreconditioned 2-norm); the iteration count is the number of products with K
inside the loop.  alpha and beta are recorded, from which the Lanczos tridiagonal gives an
estimate of the extreme eigenvalues of P K.
"""
from __future__ import annotations

import numpy as np

from .direct import factorized


class Schwarz:
    def __init__(self, dec, coarse=None, factor="superlu"):
        self.dec = dec
        self.coarse = coarse
        K = dec.prob.K
        self.solves = [factorized(K[Ij][:, Ij], factor) for Ij in dec.I]

    def apply(self, r):
        z = np.zeros_like(r)
        for Ij, solve in zip(self.dec.I, self.solves):
            z[Ij] += solve(r[Ij])
        if self.coarse is not None:
            z += self.coarse.apply(r)
        return z


def pcg(K, b, M=None, rtol=1e-8, maxit=1000, x0=None):
    """Returns x, iterations, relative residual history, (alphas, betas)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - K @ x if x0 is not None else b.copy()
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / nb]
    alphas, betas = [], []
    if hist[-1] <= rtol:
        return x, 0, np.array(hist), (alphas, betas)
    z = M(r) if M is not None else r.copy()
    p = z.copy()
    rz = r @ z
    it = 0
    while it < maxit:
        q = K @ p
        it += 1
        pq = p @ q
        if not (pq > 0):
            raise FloatingPointError("CG breakdown: p^T K p <= 0")
        a = rz / pq
        x += a * p
        r -= a * q
        alphas.append(a)
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= rtol:
            break
        z = M(r) if M is not None else r.copy()
        rz_new = r @ z
        beta = rz_new / rz
        betas.append(beta)
        p = z + beta * p
        rz = rz_new
    return x, it, np.array(hist), (alphas, betas)


def lanczos_extremes(alphas, betas):
    """Extreme eigenvalues of the CG Lanczos tridiagonal (estimate of spec(P K))."""
    k = len(alphas)
    if k == 0:
        return np.nan, np.nan
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1.0 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i + 1 < k and i < len(betas):
            T[i, i + 1] = T[i + 1, i] = np.sqrt(betas[i]) / alphas[i]
    ev = np.linalg.eigvalsh(T)
    return ev[0], ev[-1]


def solve(cfg, prob=None, one_level=False, rtol=None, dense_eigen=None, maxit=2000,
          factor="superlu", progress=None):
    """Full oracle pipeline for a laminate descriptor; returns a dict of results.
    factor: direct method of the subdomain and eigensolver factorisations (direct.py)."""
    from .dd import Decomposition, box_partition
    from .fem import Problem
    from .geneo import Coarse
    s = cfg["solver"]
    prob = prob or Problem(cfg)
    part = box_partition(prob.mesh, s["px"], s["py"])
    dec = Decomposition(prob, part, s["overlap"])
    coarse = None if one_level else Coarse(dec, nev=s["nev"] or 0, tau=s["tau"] or 0.1,
                                           nev_max=s["nev_max"], dense=dense_eigen,
                                           factor=factor, progress=progress)
    P = Schwarz(dec, coarse, factor=factor)
    x, it, hist, ab = pcg(prob.K, prob.f, P.apply, rtol=rtol or s["rtol"], maxit=maxit)
    return dict(prob=prob, dec=dec, coarse=coarse, P=P, x=x, iters=it, hist=hist,
                alphas=ab[0], betas=ab[1])

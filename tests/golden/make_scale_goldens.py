"""Writes the stored oracle results of the large parity cases.

    python tests/golden/make_scale_goldens.py flat32     # about an hour on 8 cores
    python tests/golden/make_scale_goldens.py lsec60

Calls only the oracle (and the seeded inputs of `workloads`); nothing here comes from the
GPU library.  Vectors too large to store are kept at seeded sample positions plus their
norm.  Cases:

* flat32: the 3M-DOF flat laminate reduced to 32 x 32 x 59 elements and 4 x 4 subdomains
  (overlap 2, GenEO threshold 0.1): GenEO modes and eigenvalues per subdomain, the
  two-level preconditioner applied to a seeded vector, the PCG trajectory and solution at
  rtol 1e-8 (trajectory parity, section 2.3 / Eq. eq-pre);
* lsec60: the curved wrinkled L-section of the 3M-DOF target reduced to 60 x 6 x 59
  elements and 8 x 2 subdomains: GenEO modes and eigenvalues, and the solution of K u = f
  by the oracle's PCG to rtol 1e-12 (the discrete solution, for the FP64 and mixed paths),
  with the oracle's own sensitivity to assembly rounding: K summed in reverse element order
  and solved again (any two FP64 assemblies of K differ by that much, times kappa(K)).

Local and eigensolver factorisations use LAPACK banded Cholesky (oracle/direct.py).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import pcg  # noqa: E402

SEED_R = 8401          # seeded vector for P r
NSAMPLE = 4096


def log(msg, t0=[time.time()]):
    print(f"[{time.time() - t0[0]:7.1f} s] {msg}", flush=True)


def run(name, cfg, rtol, extra_rtol=None):
    log(f"{name}: building the problem")
    from oracle.fem import Problem
    prob = Problem(cfg)
    log(f"{name}: {prob.n} free DOFs")
    R = pcg.solve(cfg, prob=prob, rtol=rtol, factor="band", progress=log)
    log(f"{name}: {R['iters']} PCG iterations to rtol {rtol}")
    co, dec = R["coarse"], R["dec"]
    n_full = prob.mesh.n_dofs
    free = prob.free
    idx = workloads.sample_indices(n_full, NSAMPLE)
    idx = idx[free[idx]]                              # free DOFs only
    pos = np.cumsum(free) - 1                         # full index -> free position
    r_full = workloads.seeded_vector(n_full, SEED_R) * free
    z = R["P"].apply(r_full[free])
    x = R["x"]
    out = dict(n_dofs=n_full, n_free=prob.n, n0=co.n0, nev=np.array(co.nev),
               lam=np.concatenate([np.asarray(l) for l in co.lams]),
               iters=R["iters"], hist=R["hist"], idx=idx,
               Pr=z[pos[idx]], Pr_norm=np.linalg.norm(z), Pr_maxabs=np.abs(z).max(),
               x=x[pos[idx]], x_norm=np.linalg.norm(x), rtol=rtol, seed_r=SEED_R,
               n_interior=np.array([len(I) for I in dec.I]))
    if extra_rtol:
        xt, it2, h2, _ = pcg.pcg(prob.K, prob.f, R["P"].apply, rtol=extra_rtol, maxit=4000)
        log(f"{name}: {it2} PCG iterations to rtol {extra_rtol}")
        out.update(x_tight=xt[pos[idx]], x_tight_norm=np.linalg.norm(xt),
                   tight_rtol=extra_rtol, tight_iters=it2)
        # sensitivity of the discrete solution to the rounding of assembly: K summed over the
        # elements in reverse order (the same matrix up to rounding) and solved again
        from oracle.fem import assemble
        Kr = assemble(prob.mesh, prob.Ke, elems=np.arange(prob.mesh.n_elems)[::-1])
        Kr = Kr[prob.free][:, prob.free].tocsr()
        nd = int((Kr != prob.K).nnz)
        xr, it3, _, _ = pcg.pcg(Kr, prob.f, R["P"].apply, rtol=extra_rtol, maxit=4000)
        d = float(np.linalg.norm(xr - xt) / np.linalg.norm(xt))
        log(f"{name}: reverse-order assembly differs in {nd} entries; its solution differs by "
            f"{d:.3e} ({it3} iterations)")
        out.update(reorder_entries=nd, reorder_diff=d,
                   reorder_sample_diff=float(np.linalg.norm(xr[pos[idx]] - xt[pos[idx]]) /
                                             np.linalg.norm(xt[pos[idx]])))
    path = os.path.join(HERE, f"scale_{name}.npz")
    np.savez_compressed(path, **out)
    log(f"{name}: wrote {path}")


if __name__ == "__main__":
    which = sys.argv[1:] or ["lsec60", "flat32"]
    for w in which:
        if w == "flat32":
            run("flat32", workloads.cfg1(nx=32, ny=32, px=4, py=4), rtol=1e-8)
        elif w == "lsec60":
            run("lsec60", workloads.cfg2(nx=60, ny=6, px=8, py=2), rtol=1e-8,
                extra_rtol=1e-12)
        else:
            sys.exit(f"unknown case {w}")

"""Pins of the oracle's periodic boundary conditions across the width (section 3: periodic
conditions at the free edge model a very wide part; section 2.1 lists periodic conditions
among the module's features).

* the unconstrained periodic K has exactly four zero-energy modes: the three translations and
  the rotation about the periodic axis (the other two rotations are not periodic);
* under a load that does not vary across the width, the periodic solution does not vary
  along l either (every lattice line along l carries one displacement), although the ply
  angles break the mirror symmetry and the non-periodic solution does vary;
* doubling the period (twice the width and elements) leaves that solution unchanged;
* on a wrinkled, defected L-section (defect centred across the width, so the geometry is
  periodic) the periodic K is SPD after the clamp and holds the four periodic modes.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import fem
from oracle.mesh import Mesh


def _periodic(cfg):
    cfg = dict(cfg)
    cfg["periodic"] = True
    return cfg


def _modes(xyz, which):
    out = []
    for c in range(3):
        t = np.zeros_like(xyz)
        t[:, c] = 1
        out.append(t.ravel())
    for axis in which:
        out.append(np.cross(np.eye(3)[axis], xyz).ravel())
    return np.array(out)


def test_periodic_null_space_is_four_dimensional():
    cfg = _periodic(workloads.small_flat(nx=2, ny=3, length=2.0, width=3.0))
    mesh = Mesh(cfg)
    K = fem.assemble(mesh, fem.all_element_matrices(mesh)).toarray()
    ev = np.linalg.eigvalsh(K)
    assert int(np.sum(ev < 1e-10 * ev[-1])) == 4
    nK = np.abs(K).max()
    for r in _modes(mesh.xyz, [1]):                        # rotation about y is periodic
        assert np.linalg.norm(K @ r) <= 1e-11 * nK * np.linalg.norm(r)
    for r in _modes(mesh.xyz, [0, 2])[3:]:                 # about x and z it is not
        assert np.linalg.norm(K @ r) > 1e-6 * nK * np.linalg.norm(r)


def _solve(cfg):
    prob = fem.Problem(cfg)
    return prob, prob.to_full(spla.spsolve(prob.K.tocsc(), prob.f))


def _lines(mesh, u):
    """Displacements grouped by lattice line along l: {(i2, k2, j2 parity): [u, ...]}."""
    U = u.reshape(-1, 3)
    g = {}
    for n, (i2, j2, k2) in enumerate(mesh.lat):
        g.setdefault((i2, k2, j2 % 2), []).append(U[n])
    return {k: np.array(v) for k, v in g.items()}


def test_periodic_solution_is_invariant_along_the_width():
    layers = [{"mat": "ply", "t": 0.25, "nel": 2, "angle": 45.0},
              {"mat": "resin", "t": 0.05, "nel": 1, "angle": 0.0},
              {"mat": "ply", "t": 0.25, "nel": 2, "angle": -30.0}]
    base = workloads.small_flat(nx=4, ny=3, layers=layers, length=4.0, width=3.0)
    prob, u = _solve(_periodic(base))
    scale = np.abs(u).max()
    for pts in _lines(prob.mesh, u).values():
        assert np.abs(pts - pts[0]).max() <= 1e-10 * scale
    # the free-edge solution of the same plate does vary across the width
    prob0, u0 = _solve(base)
    dev = max(np.abs(p - p[0]).max() for p in _lines(prob0.mesh, u0).values())
    assert dev > 1e-4 * np.abs(u0).max()
    # doubling the period leaves the solution unchanged
    wide = workloads.small_flat(nx=4, ny=6, layers=layers, length=4.0, width=6.0)
    prob2, u2 = _solve(_periodic(wide))
    L1, L2 = _lines(prob.mesh, u), _lines(prob2.mesh, u2)
    assert L1.keys() == L2.keys()
    for k in L1:
        assert np.abs(L2[k] - L1[k][0]).max() <= 1e-10 * scale


def test_periodic_defected_lsection():
    cfg = _periodic(workloads.defect_lsection(nx=16, ny=4, d=0.3))
    mesh = Mesh(cfg)
    # the nodes of the wrapped plane are the ones at l = 0
    assert mesh.n_nodes < Mesh(workloads.defect_lsection(nx=16, ny=4, d=0.3)).n_nodes
    K = fem.assemble(mesh, fem.all_element_matrices(mesh))
    nK = spla.norm(K)
    for r in _modes(mesh.xyz, [1]):
        assert np.linalg.norm(K @ r) <= 1e-11 * nK * np.linalg.norm(r)
    free = mesh.free_mask()
    np.linalg.cholesky(K[free][:, free].toarray())

"""Overlapping domain decomposition (oracle; test infrastructure).

Section 2.3 (Fig. fig-domaindecomp): the mesh is split into subdomains of roughly equal size
that overlap by whole layers of elements; the local problems carry zero-displacement
conditions on the artificial subdomain boundaries, and local modes are glued by a partition
of unity.

Readings where the paper is silent:

* core partition: P_x x P_y in-plane boxes of element index ranges, full thickness; box p
  along an axis of n elements covers [floor(p n / P), floor((p + 1) n / P));
* overlap growth: Omega^(l+1) = Omega^(l) plus every element sharing a node with it;
* interior DOFs I_j: free DOFs of nodes all of whose elements lie in Omega_j (this is the
  zero-displacement condition on the artificial boundary);
* partition of unity: X_j = 1 / (number of subdomains whose I_k holds the DOF), on I_j.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def box_partition(mesh, px, py):
    ex, ey = mesh.eidx[:, 0], mesh.eidx[:, 1]
    bx = np.array([(p * mesh.nx) // px for p in range(px + 1)])
    by = np.array([(p * mesh.ny) // py for p in range(py + 1)])
    ix = np.searchsorted(bx, ex, side="right") - 1
    iy = np.searchsorted(by, ey, side="right") - 1
    return (iy * px + ix).astype(np.int64)


def incidence(mesh):
    """Element-node incidence matrix (n_elems x n_nodes, 0/1)."""
    E = mesh.n_elems
    rows = np.repeat(np.arange(E), 20)
    return sp.csr_matrix((np.ones(E * 20), (rows, mesh.conn.ravel())),
                         shape=(E, mesh.n_nodes))


class Decomposition:
    def __init__(self, prob, part, overlap):
        mesh = prob.mesh
        self.prob = prob
        self.n_sub = int(part.max()) + 1
        inc = incidence(mesh)
        incT = inc.T.tocsr()
        n_adj = np.asarray(incT.sum(axis=1)).ravel()          # elements per node
        self.elems, self.interior_nodes, self.touch_nodes = [], [], []
        for j in range(self.n_sub):
            om = (part == j).astype(np.float64)
            for _ in range(overlap):
                touched = (incT @ om) > 0
                om = ((inc @ touched.astype(np.float64)) > 0).astype(np.float64)
            in_om = om > 0
            self.elems.append(np.nonzero(in_om)[0])
            cnt = incT @ om
            self.interior_nodes.append(np.nonzero(cnt == n_adj)[0])
            self.touch_nodes.append(np.nonzero(cnt > 0)[0])
        # free-DOF index sets (positions in the free numbering)
        full_to_free = -np.ones(mesh.n_dofs, dtype=np.int64)
        full_to_free[prob.free_idx] = np.arange(prob.n)
        self.full_to_free = full_to_free

        def dofs_of(nodes):
            d = (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()
            f = full_to_free[d]
            return f[f >= 0]

        self.I = [dofs_of(n) for n in self.interior_nodes]
        self.D = [dofs_of(n) for n in self.touch_nodes]
        mult = np.zeros(prob.n)
        for Ij in self.I:
            mult[Ij] += 1.0
        if (mult == 0).any():
            raise ValueError("some free DOF lies in no subdomain interior (overlap >= 1?)")
        self.mult = mult
        self.X = [1.0 / mult[Ij] for Ij in self.I]
        # overlap elements: in Omega_j and in some other Omega_k
        cover = np.zeros(mesh.n_elems)
        for e in self.elems:
            cover[e] += 1
        self.overlap_elems = [e[cover[e] > 1] for e in self.elems]

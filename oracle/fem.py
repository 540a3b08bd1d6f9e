"""Global stiffness and load of K u = f (Eq. eq-1), oracle.

K is assembled from element matrices (section 2.1) as a plain sum over elements; the
clamped end (all three displacement components of every node on the s = s_min face,
section 2.2 "fixing all degrees of freedom on the other limb") is removed from the system,
leaving the free DOFs in canonical order (DOF = 3 * node + component).

Loads (readings): a uniform traction t0 on the s = s_max end face, or a pure end moment
per unit width M applied as the linear normal traction
t = -12 M (zeta - T/2) / T^3 * n_out, whose force resultant vanishes and whose moment about
the mid-thickness line is M per unit width; the sign puts the inner face (zeta = 0) in
tension along the limb, which opens a corner (section 2.2 corner unfolding).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .element import element_stiffness, face_load
from .material import layer_material
from .mesh import Mesh, total_thickness


def element_data(mesh):
    Cs, angs = layer_material(mesh.cfg)
    X = mesh.elem_coords()
    return X, Cs[mesh.elayer], angs[mesh.elayer]


def all_element_matrices(mesh, nq=3):
    X, C, a = element_data(mesh)
    return element_stiffness(X, C, a, nq=nq)


def element_dofs(mesh):
    return (3 * mesh.conn[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 60)


def assemble(mesh, Ke, elems=None, n=None):
    """Sum_e P_e^T K_e P_e over the given elements (all DOFs, no boundary conditions)."""
    if elems is None:
        elems = np.arange(mesh.n_elems)
    n = mesh.n_dofs if n is None else n
    d = element_dofs(mesh)[elems]
    rows = np.repeat(d, 60, axis=1).ravel()
    cols = np.tile(d, (1, 60)).ravel()
    vals = Ke[elems].reshape(len(elems), -1).ravel()
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def load_vector(mesh):
    """Consistent nodal loads on all DOFs (Eq. eq-1 right-hand side)."""
    f = np.zeros(mesh.n_dofs, dtype=mesh.xyz.dtype)
    le = mesh.load_elements()
    X = mesh.elem_coords(le)
    load = mesh.cfg["load"]
    if load["kind"] == "traction":
        t0 = np.array(load["t0"], dtype=float)
        fe = face_load(X, 1.0, lambda x, n: np.broadcast_to(t0, x.shape).copy())
    else:
        T = total_thickness(mesh.cfg)
        k = -12.0 * load["M"] / T ** 3
        # through-thickness parameter at the face points, interpolated from the nodes
        Zp = mesh.param[mesh.conn[le], 2]
        Zx = np.concatenate([X, Zp[:, :, None]], axis=2)    # carry zeta as a 4th "coordinate"
        fe = _face_load_with_param(Zx, k, T)
    d = element_dofs(mesh)[le]
    np.add.at(f, d.ravel(), fe.ravel())
    return f


def _face_load_with_param(Zx, k, T):
    from .element import gauss_1d, shape
    x1, w1 = gauss_1d(3)
    pts = np.array([(1.0, x1[i], x1[j]) for j in range(3) for i in range(3)])
    wts = np.array([w1[i] * w1[j] for j in range(3) for i in range(3)])
    N, dN = shape(pts)
    X = Zx[:, :, :3]
    zeta = np.einsum("qa,ea->eq", N, Zx[:, :, 3])
    t_eta = np.einsum("qa,eai->eqi", dN[:, :, 1], X)
    t_zt = np.einsum("qa,eai->eqi", dN[:, :, 2], X)
    nvec = np.cross(t_eta, t_zt)
    dA = np.sqrt(np.sum(nvec * nvec, axis=-1))
    nout = nvec / dA[..., None]
    t = (k * (zeta - 0.5 * T))[..., None] * nout
    f = np.einsum("qa,eqi,eq->eai", N, t, dA * wts[None, :])
    return f.reshape(Zx.shape[0], 60)


class Problem:
    """Mesh, element matrices, K_ff and f_f of one laminate configuration."""

    def __init__(self, cfg, nq=3):
        self.cfg = cfg
        self.mesh = Mesh(cfg)
        self.Ke = all_element_matrices(self.mesh, nq=nq)
        self.K_all = assemble(self.mesh, self.Ke)
        self.f_all = load_vector(self.mesh)
        self.free = self.mesh.free_mask()
        self.free_idx = np.nonzero(self.free)[0]
        self.K = self.K_all[self.free][:, self.free].tocsr()
        self.f = self.f_all[self.free]
        self.n = self.K.shape[0]

    def to_full(self, u_free):
        u = np.zeros(self.mesh.n_dofs, dtype=np.result_type(u_free, 1.0))
        u[self.free_idx] = u_free
        return u

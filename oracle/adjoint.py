"""Gradient of a through-thickness stress functional by the adjoint method (oracle; test
infrastructure).

The paper's corner-unfolding study is governed by the through-thickness normal stress
sigma_33 in the curved region (section 3).  The functional is

    J(u, p) = sum over the region's elements and Gauss points of sigma_33^2 det J w,

with sigma_33 = e3 . sigma e3, sigma = C_g B u_e the stress in global axes and e3 the
laminate normal of the local frame (region: the arc elements of an L-section, every
element of a flat part).  With K lambda = dJ/du on the free DOFs,

    dJ/dp = dJ/dp|_u - lambda^T (dK/dp u - df/dp).

The partial derivatives with respect to the wrinkle amplitude A and wavelength L_w (through
the node coordinates) and the modulus E11 of a layer (through its stiffness) are taken by
complex-step differentiation (Squire and Trapp 1998) of this oracle's own mesh, element,
load and objective routines, which is exact to rounding: f(p + i h) = f(p) + i h f'(p) +
O(h^2).  Everything is FP64 with direct solves (SuperLU).
"""
from __future__ import annotations

import copy

import numpy as np
import scipy.sparse.linalg as spla

from .element import gauss_point_data, local_frame, material_at_points, strain_matrix
from .fem import Problem, element_data, element_dofs, load_vector
from .material import layer_material
from .mesh import Mesh

H = 1e-30                        # complex step


def region_elements(mesh):
    return mesh.arc_elements()


def sigma33(mesh, u_full, elems, layer_C=None):
    """sigma_33 (E, Q) at the Gauss points of `elems` and det J w (E, Q)."""
    X, C, ang = element_data(mesh)
    if layer_C is not None:
        C = layer_C[mesh.elayer]
    X, C, ang = X[elems], C[elems], ang[elems]
    gp = gauss_point_data(X)
    Cq = material_at_points(gp["J"], C, ang)
    B = strain_matrix(gp["G"])
    ue = u_full[element_dofs(mesh)[elems]]
    sig = np.einsum("eqIJ,eqJb,eb->eqI", Cq, B, ue)
    e3 = local_frame(gp["J"])[..., 2, :]
    n1, n2, n3 = e3[..., 0], e3[..., 1], e3[..., 2]
    s33 = (sig[..., 0] * n1 * n1 + sig[..., 1] * n2 * n2 + sig[..., 2] * n3 * n3 +
           2 * (sig[..., 3] * n2 * n3 + sig[..., 4] * n1 * n3 + sig[..., 5] * n1 * n2))
    return s33, gp["detJ"] * gp["w"][None, :]


def objective(mesh, u_full, layer_C=None):
    els = region_elements(mesh)
    s33, dv = sigma33(mesh, u_full, els, layer_C)
    return np.sum(s33 * s33 * dv)


def objective_grad(mesh, u_full):
    """dJ/du on all DOFs: J is quadratic, J = sum (a^T C_g B u_e)^2 dv."""
    els = region_elements(mesh)
    X, C, ang = element_data(mesh)
    X, C, ang = X[els], C[els], ang[els]
    gp = gauss_point_data(X)
    Cq = material_at_points(gp["J"], C, ang)
    B = strain_matrix(gp["G"])
    e3 = local_frame(gp["J"])[..., 2, :]
    n1, n2, n3 = e3[..., 0], e3[..., 1], e3[..., 2]
    a = np.stack([n1 * n1, n2 * n2, n3 * n3, 2 * n2 * n3, 2 * n1 * n3, 2 * n1 * n2], axis=-1)
    row = np.einsum("eqI,eqIJ,eqJb->eqb", a, Cq, B)          # d sigma_33 / d u_e
    dofs = element_dofs(mesh)[els]
    s33 = np.einsum("eqb,eb->eq", row, u_full[dofs])
    dv = gp["detJ"] * gp["w"][None, :]
    ge = np.einsum("eq,eqb->eb", 2 * s33 * dv, row)
    g = np.zeros(mesh.n_dofs)
    np.add.at(g, dofs.ravel(), ge.ravel())
    return g


def _element_energy_im(mesh_c, u_full, lam_full, elems, layer_C=None):
    """Im(lambda_e^T K_e(p + i h) u_e) / h summed over `elems`."""
    from .element import element_stiffness
    X, C, ang = element_data(mesh_c)
    if layer_C is not None:
        C = layer_C[mesh_c.elayer]
    Ke = element_stiffness(X[elems], C[elems], ang[elems])
    d = element_dofs(mesh_c)[elems]
    return np.einsum("ea,eab,eb->", lam_full[d], Ke, u_full[d]).imag / H


def gradient(cfg, prob=None):
    """J and dJ/dp = [dA, dL_w, dE11 of every layer] for the exact solution of K u = f."""
    prob = prob or Problem(cfg)
    mesh = prob.mesh
    lu = spla.splu(prob.K.tocsc())
    u = prob.to_full(lu.solve(prob.f))
    g = objective_grad(mesh, u)[prob.free]
    lam = prob.to_full(lu.solve(g))
    J = objective(mesh, u)
    allel = np.arange(mesh.n_elems)
    out = np.zeros(2 + len(cfg["layers"]))
    A, Lw = cfg.get("wrinkle", (0.0, 1.0))
    for p in range(2):
        cc = copy.deepcopy(cfg)
        cc["wrinkle"] = (A + 1j * H, Lw) if p == 0 else (A, Lw + 1j * H)
        mc = Mesh(cc)
        dK = _element_energy_im(mc, u, lam, allel)
        df = lam[prob.free] @ (load_vector(mc).imag / H)[prob.free]
        dJ = objective(mc, u).imag / H
        out[p] = dJ - (dK - df)
    C0, _ = layer_material(cfg)
    for k, L in enumerate(cfg["layers"]):
        cc = copy.deepcopy(cfg)
        key = "E1" if L["mat"] == "ply" else "E"
        from workloads import PLY, RESIN
        base = L.get(key, PLY["E1"] if L["mat"] == "ply" else RESIN["E"])
        cc["layers"][k][key] = base + 1j * H
        Cc, _ = layer_material(cc)
        els = np.nonzero(mesh.elayer == k)[0]
        dK = _element_energy_im(mesh, u, lam, els, layer_C=Cc) if len(els) else 0.0
        dJ = objective(mesh, u, layer_C=Cc).imag / H
        out[2 + k] = dJ - dK
    return dict(J=J, dJdp=out, u=u, lam=lam, prob=prob)


def objective_at(cfg):
    """J of the exact solution for the descriptor (finite-difference checks)."""
    prob = Problem(cfg)
    u = prob.to_full(spla.spsolve(prob.K.tocsc(), prob.f))
    return objective(prob.mesh, u)

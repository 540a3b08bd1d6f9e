"""20-node serendipity hexahedron with full 3x3x3 Gauss integration (oracle).

Section 2.1: a 20-node serendipity element with nodes at the 8 vertices and on the 12
edges, fully integrated (as opposed to the reduced integration of the comparison element,
section 2.2).  "Full integration" is read as the 3x3x3 Gauss-Legendre rule.

The element stiffness is K_e = sum_q B_q^T C_q B_q det(J_q) w_q with the material stiffness
C_q rotated into the local frame at each Gauss point (reading, the paper being silent):
e1 = unit dx/dxi, e2 = unit component of dx/deta orthogonal to e1, e3 = e1 x e2, and the
ply fibre rotated by the ply angle about e3.
"""
from __future__ import annotations

import numpy as np

from .material import ply_axes, rotate_stiffness
from .mesh import reference_nodes


def gauss_1d(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def gauss_hex(n=3):
    x, w = gauss_1d(n)
    pts, wts = [], []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                pts.append((x[i], x[j], x[k]))
                wts.append(w[i] * w[j] * w[k])
    return np.array(pts), np.array(wts)


def shape(p):
    """Serendipity shape functions N (npts, 20) and reference gradients (npts, 20, 3)."""
    p = np.atleast_2d(p)
    ref = reference_nodes()
    xi, eta, zt = p[:, 0:1], p[:, 1:2], p[:, 2:3]
    a, b, c = ref[None, :, 0], ref[None, :, 1], ref[None, :, 2]
    N = np.zeros((p.shape[0], 20))
    dN = np.zeros((p.shape[0], 20, 3))
    vert = (a != 0) & (b != 0) & (c != 0)
    # vertices: 1/8 (1+xi a)(1+eta b)(1+zt c)(xi a + eta b + zt c - 2)
    fx, fy, fz = 1 + xi * a, 1 + eta * b, 1 + zt * c
    g = xi * a + eta * b + zt * c - 2
    Nv = 0.125 * fx * fy * fz * g
    dNv_x = 0.125 * (a * fy * fz * g + fx * fy * fz * a)
    dNv_y = 0.125 * (b * fx * fz * g + fx * fy * fz * b)
    dNv_z = 0.125 * (c * fx * fy * g + fx * fy * fz * c)
    # edge nodes with xi_a = 0: 1/4 (1 - xi^2)(1 + eta b)(1 + zt c), and permutations
    ex_, ey_, ez_ = (a == 0), (b == 0), (c == 0)
    Nex = 0.25 * (1 - xi ** 2) * fy * fz
    Ney = 0.25 * (1 - eta ** 2) * fx * fz
    Nez = 0.25 * (1 - zt ** 2) * fx * fy
    N = np.where(vert, Nv, np.where(ex_, Nex, np.where(ey_, Ney, Nez)))
    dx = np.where(vert, dNv_x,
                  np.where(ex_, 0.25 * (-2 * xi) * fy * fz,
                           np.where(ey_, 0.25 * (1 - eta ** 2) * a * fz,
                                    0.25 * (1 - zt ** 2) * a * fy)))
    dy = np.where(vert, dNv_y,
                  np.where(ex_, 0.25 * (1 - xi ** 2) * b * fz,
                           np.where(ey_, 0.25 * (-2 * eta) * fx * fz,
                                    0.25 * (1 - zt ** 2) * fx * b)))
    dz = np.where(vert, dNv_z,
                  np.where(ex_, 0.25 * (1 - xi ** 2) * fy * c,
                           np.where(ey_, 0.25 * (1 - eta ** 2) * fx * c,
                                    0.25 * (-2 * zt) * fx * fy)))
    dN[:, :, 0], dN[:, :, 1], dN[:, :, 2] = dx, dy, dz
    return N, dN


def local_frame(J):
    """Orthonormal frame (e1, e2, e3) from the Jacobian columns dx/dxi and dx/deta."""
    t1 = J[..., :, 0]
    t2 = J[..., :, 1]
    # lengths as sqrt(sum x^2) (not abs): analytic, so complex-step derivatives go through
    e1 = t1 / np.sqrt(np.sum(t1 * t1, axis=-1, keepdims=True))
    v = t2 - np.sum(t2 * e1, axis=-1, keepdims=True) * e1
    e2 = v / np.sqrt(np.sum(v * v, axis=-1, keepdims=True))
    e3 = np.cross(e1, e2)
    return np.stack([e1, e2, e3], axis=-2)


def strain_matrix(G):
    """B (..., 6, 60) from shape gradients G (..., 20, 3); Voigt [11,22,33,23,13,12]."""
    B = np.zeros(G.shape[:-2] + (6, 60), dtype=G.dtype)
    gx, gy, gz = G[..., 0], G[..., 1], G[..., 2]
    B[..., 0, 0::3] = gx
    B[..., 1, 1::3] = gy
    B[..., 2, 2::3] = gz
    B[..., 3, 1::3] = gz
    B[..., 3, 2::3] = gy
    B[..., 4, 0::3] = gz
    B[..., 4, 2::3] = gx
    B[..., 5, 0::3] = gy
    B[..., 5, 1::3] = gx
    return B


def gauss_point_data(X, nq=3):
    """Jacobians, determinants, physical gradients and weights at the Gauss points."""
    pts, wts = gauss_hex(nq)
    N, dN = shape(pts)
    J = np.einsum("eai,qaj->eqij", X, dN)           # J_ij = dx_i / dxi_j
    detJ = np.linalg.det(J)
    Jinv = np.linalg.inv(J)                            # Jinv_ji = dxi_j / dx_i
    G = np.einsum("qaj,eqji->eqai", dN, Jinv)          # dN_a / dx_i
    return dict(N=N, J=J, detJ=detJ, G=G, w=wts)


def material_at_points(J, Cloc, angle):
    """Rotated stiffness C_q (E, Q, 6, 6) at every Gauss point."""
    frame = local_frame(J)
    Q = ply_axes(frame, np.broadcast_to(angle[:, None], J.shape[:2]))
    return rotate_stiffness(np.broadcast_to(Cloc[:, None], J.shape[:2] + (6, 6)), Q)


def element_stiffness(X, Cloc, angle, nq=3, chunk=512):
    """K_e for elements with nodes X (E, 20, 3), material Cloc (E, 6, 6), ply angle (E,)."""
    X = np.asarray(X)
    out = np.empty((X.shape[0], 60, 60), dtype=np.result_type(X, Cloc))
    for s in range(0, X.shape[0], chunk):
        sl = slice(s, s + chunk)
        gp = gauss_point_data(X[sl], nq)
        Cq = material_at_points(gp["J"], Cloc[sl], angle[sl])
        B = strain_matrix(gp["G"])
        CB = np.einsum("eqIJ,eqJb->eqIb", Cq, B)
        K = np.einsum("eqIa,eqIb,eq->eab", B, CB, gp["detJ"] * gp["w"][None, :])
        out[sl] = 0.5 * (K + np.swapaxes(K, 1, 2))
    return out


def face_load(X, face_xi, traction_fn, nq=3):
    """Consistent nodal loads (E, 60) of a traction on the local face xi = face_xi.

    traction_fn(x, n_out) -> traction vector, where x are physical points (E, Q, 3) and
    n_out the outward unit normals.  f_a = int N_a t dA with a 3x3 Gauss rule on the face.
    """
    x1, w1 = gauss_1d(nq)
    pts = np.array([(face_xi, x1[i], x1[j]) for j in range(nq) for i in range(nq)])
    wts = np.array([w1[i] * w1[j] for j in range(nq) for i in range(nq)])
    N, dN = shape(pts)
    xq = np.einsum("qa,eai->eqi", N, X)
    t_eta = np.einsum("qa,eai->eqi", dN[:, :, 1], X)
    t_zt = np.einsum("qa,eai->eqi", dN[:, :, 2], X)
    nvec = np.cross(t_eta, t_zt) * np.sign(face_xi)
    dA = np.sqrt(np.sum(nvec * nvec, axis=-1))
    nout = nvec / dA[..., None]
    t = traction_fn(xq, nout)
    f = np.einsum("qa,eqi,eq->eai", N, t, dA * wts[None, :])
    return f.reshape(X.shape[0], 60)

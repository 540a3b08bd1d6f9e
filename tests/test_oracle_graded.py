"""Pins of the oracle's graded, edge-treated meshes (section 2.2: bias ratios 400 across the
width and 10 through each layer, resin edge strips, a stiff end layer; section 3.1: bias 2
towards the defect).

* grading: element sizes along each graded direction are symmetric, monotone towards the
  refined ends, sum to the segment, and their largest-to-smallest ratio is the bias;
* materials: the elements across the strips carry the resin-edge material of Table 1 and
  the loaded limb's last column the stiff material, after the layers' materials;
* the graded, edge-treated, wrinkled L-section still has the six rigid-body modes in the
  null space of its unconstrained K, and a graded plate passes the patch test;
* the paper's verification model has its printed element count and the DOF count.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import fem, material
from oracle.mesh import Mesh, graded, l_boundaries, s_boundaries, zeta_boundaries


@pytest.mark.parametrize("n,bias,fine", [(48, 400.0, "ends"), (7, 10.0, "ends"),
                                         (6, 10.0, "ends"), (38, 2.0, "middle"),
                                         (9, 2.0, "middle"), (1, 5.0, "ends")])
def test_graded_sizes(n, bias, fine):
    b = graded(n, bias, fine)
    h = np.diff(b)
    assert abs(b[0]) == 0.0 and abs(b[-1] - 1.0) < 1e-15
    assert np.allclose(h, h[::-1], rtol=1e-12)
    if n > 2:
        assert abs(h.max() / h.min() - bias) < 1e-9 * bias
        half = h[: (n + 1) // 2]
        d = np.diff(half)
        assert np.all(d > 0) if fine == "ends" else np.all(d < 0)
    else:
        assert np.allclose(h, 1.0 / n)


def test_graded_lsection_directions_and_materials():
    cfg = workloads.graded_lsection(nx=20, ny=8)
    m = Mesh(cfg)
    # across the width: strips uniform, laminate graded towards its two edges
    lb = l_boundaries(cfg)
    st = cfg["edge_strip"]
    assert abs(lb[st["ny"]] - st["width"]) < 1e-14
    assert abs(lb[-1 - st["ny"]] - (cfg["width"] - st["width"])) < 1e-14
    h = np.diff(lb[st["ny"]:len(lb) - st["ny"]])
    assert abs(h.max() / h.min() - cfg["bias"]["l"]) < 1e-9 * cfg["bias"]["l"]
    # through each layer
    zb, lay = zeta_boundaries(cfg)
    for li in range(len(cfg["layers"])):
        hz = np.diff(zb)[lay == li]
        if len(hz) > 2:
            assert abs(hz.max() / hz.min() - cfg["bias"]["z"]) < 1e-9 * cfg["bias"]["z"]
        assert abs(hz.sum() - cfg["layers"][li]["t"]) < 1e-15
    # along the arc: finest at mid-arc, the limbs uniform
    sb = s_boundaries(cfg)
    nl = cfg["nx_limb"]
    ha = np.diff(sb[nl:len(sb) - nl])
    assert abs(ha.max() / ha.min() - cfg["bias"]["s"]) < 1e-9 * cfg["bias"]["s"]
    assert np.allclose(np.diff(sb[: nl + 1]), cfg["limb"] / nl, rtol=1e-12)
    # materials: the layers, then the edge resin, then the stiff end
    C, ang = material.layer_material(cfg)
    nlay = len(cfg["layers"])
    assert len(C) == nlay + 2
    lam_e = material.isotropic_stiffness(workloads.RESIN_EDGE["E"], workloads.RESIN_EDGE["nu"])
    lam_s = material.isotropic_stiffness(workloads.STIFF_END["E"], workloads.STIFF_END["nu"])
    assert np.allclose(C[nlay], lam_e, rtol=1e-12) and np.allclose(C[nlay + 1], lam_s, rtol=1e-12)
    ex, ey = m.eidx[:, 0], m.eidx[:, 1]
    strip = (ey < st["ny"]) | (ey >= cfg["ny"] - st["ny"])
    assert np.all(m.elayer[(ex == cfg["nx"] - 1)] == nlay + 1)
    assert np.all(m.elayer[strip & (ex < cfg["nx"] - 1)] == nlay)
    assert np.all(m.elayer[~strip & (ex < cfg["nx"] - 1)] < nlay)


def _rbms(xyz):
    out = []
    for c in range(3):
        t = np.zeros_like(xyz)
        t[:, c] = 1
        out.append(t.ravel())
    for axis in np.eye(3):
        out.append(np.cross(axis, xyz).ravel())
    return out


def test_graded_edge_treated_lsection_rigid_body_modes():
    import scipy.sparse.linalg as spla
    cfg = workloads.graded_lsection(nx=16, ny=6, ny_strip=1)
    mesh = Mesh(cfg)
    K = fem.assemble(mesh, fem.all_element_matrices(mesh))
    nK = spla.norm(K)
    for r in _rbms(mesh.xyz):
        assert np.linalg.norm(K @ r) <= 1e-12 * nK * np.linalg.norm(r)


def test_graded_plate_patch_test():
    import scipy.sparse.linalg as spla
    layer = {"mat": "ply", "t": 0.6, "nel": 4, "angle": 25.0}
    cfg = workloads.small_flat(nx=5, ny=4, layers=[layer])
    cfg["bias"] = dict(s=3.0, l=8.0, z=5.0)
    mesh = Mesh(cfg)
    K = fem.assemble(mesh, fem.all_element_matrices(mesh)).tocsr()
    G = np.array([[1e-3, 2e-4, -3e-4], [5e-4, -7e-4, 1e-4], [2e-4, 3e-4, 9e-4]])
    u = (mesh.xyz @ G.T).ravel()
    lat = mesh.lat
    bnd = ((lat[:, 0] == 0) | (lat[:, 0] == 2 * mesh.nx) | (lat[:, 1] == 0) |
           (lat[:, 1] == 2 * mesh.ny) | (lat[:, 2] == 0) | (lat[:, 2] == 2 * mesh.nz))
    inner = np.repeat(~bnd, 3)
    Kii = K[inner][:, inner].tocsc()
    ui = spla.spsolve(Kii, -(K[inner][:, ~inner] @ u[~inner]))
    assert np.allclose(ui, u[inner], rtol=1e-9, atol=1e-13)


def test_verification_model_counts():
    cfg = workloads.verification_model()
    m = Mesh(cfg)
    assert m.n_elems == 432768
    assert 3 * m.n_nodes == 5362047
    assert abs(sum(L["t"] for L in cfg["layers"]) - 2.98) < 1e-12

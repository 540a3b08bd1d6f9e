"""Pins of the oracle's mesh, assembly and loads (sections 2.1-2.2, 3; Eq. eq-1).

* mesh counts: the verification mesh of section 2.2 (56 x 56 elements, 6 per layer over
  12 plies and 11 interfaces) has 432,768 elements, a number the paper prints;
* the six rigid-body modes lie in the null space of the unconstrained K on flat, curved and
  wrinkled meshes;
* patch test: a uniform strain is reproduced exactly on an affinely distorted mesh;
* classical lamination theory: the exact layered uniform-strain field of a flat laminate
  is reproduced, and its strain energy equals (L W / 2) eps^T A eps with the textbook A;
* loads: the traction resultant equals traction x area; the end moment has no force
  resultant and moment M W about the mid-thickness line.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import fem, material
from oracle.mesh import Mesh, total_thickness

from test_oracle_material import clt_qbar

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_verification_mesh_element_count():
    g = json.load(open(os.path.join(GOLDEN, "paper_mesh_counts.json")))
    layers = workloads.ply_layers([45, -45, 90, 0, -45, 45, -45, 45, 0, 90, 45, -45],
                                  0.23, 6, 0.02, 6)
    cfg = dict(geometry="flat", length=10.0, width=15.0, nx=56, ny=56, layers=layers)
    nz = sum(L["nel"] for L in layers)
    assert 56 * 56 * nz == g["verification_elements"]
    assert abs(total_thickness(cfg) - g["verification_thickness_mm"]) < 1e-12


def test_cfg0_sizes():
    m = Mesh(workloads.cfg0())
    assert m.n_nodes * 3 == 11691
    assert int(m.free_mask().sum()) == 10704
    assert m.n_elems == 8 * 8 * 12


def _rbms(xyz):
    out = []
    for c in range(3):
        t = np.zeros_like(xyz)
        t[:, c] = 1
        out.append(t.ravel())
    for axis in np.eye(3):
        out.append(np.cross(axis, xyz).ravel())
    return out


@pytest.mark.parametrize("cfg", [workloads.small_flat(),
                                 workloads.small_lsection(),
                                 workloads.small_lsection(amp=0.0)])
def test_rigid_body_modes_null_space(cfg):
    mesh = Mesh(cfg)
    Ke = fem.all_element_matrices(mesh)
    K = fem.assemble(mesh, Ke)
    nK = spla.norm(K)
    for r in _rbms(mesh.xyz):
        assert np.linalg.norm(K @ r) <= 1e-12 * nK * np.linalg.norm(r)
    # symmetric, and SPD once the clamp is applied
    assert spla.norm(K - K.T) <= 1e-14 * nK
    free = mesh.free_mask()
    Kf = K[free][:, free].toarray()
    np.linalg.cholesky(Kf)


def test_patch_test_affine_mesh():
    """Uniform strain on a sheared, stretched mesh of one material: exact reproduction."""
    cfg = workloads.small_flat(nx=3, ny=3, layers=[{"mat": "ply", "t": 0.6, "nel": 3,
                                                    "angle": 25.0}])
    mesh = Mesh(cfg)
    A = np.array([[1.1, 0.3, 0.05], [-0.2, 0.8, 0.1], [0.15, -0.1, 1.3]])
    mesh.xyz = mesh.xyz @ A.T
    Ke = fem.all_element_matrices(mesh)
    K = fem.assemble(mesh, Ke).tocsr()
    G = np.array([[1e-3, 2e-4, -3e-4], [5e-4, -7e-4, 1e-4], [2e-4, 3e-4, 9e-4]])
    u = (mesh.xyz @ G.T + np.array([0.1, -0.2, 0.3])).ravel()
    lat = mesh.lat
    bnd = ((lat[:, 0] == 0) | (lat[:, 0] == 2 * mesh.nx) | (lat[:, 1] == 0) |
           (lat[:, 1] == 2 * mesh.ny) | (lat[:, 2] == 0) | (lat[:, 2] == 2 * mesh.nz))
    inner = np.repeat(~bnd, 3)
    r = K @ u
    scale = abs(K) @ np.abs(u)                 # rounding scale of each row of K u
    assert np.all(np.abs(r[inner]) <= 1e-13 * scale[inner].max())
    assert np.abs(r[~inner]).max() > 1e3 * np.abs(r[inner]).max()
    # solving with the boundary values prescribed gives back the linear field
    Kii = K[inner][:, inner].tocsc()
    ui = spla.spsolve(Kii, -(K[inner][:, ~inner] @ u[~inner]))
    assert np.allclose(ui, u[inner], rtol=1e-10, atol=1e-13)


def test_classical_lamination_theory():
    angles = [0.0, 45.0, 90.0, 30.0]
    layers = workloads.ply_layers(angles, 0.25, 2, 0.05, 1)
    cfg = workloads.small_flat(nx=3, ny=2, layers=layers, length=3.0, width=2.0)
    mesh = Mesh(cfg)
    Ke = fem.all_element_matrices(mesh)
    K = fem.assemble(mesh, Ke).tocsr()
    eps = np.array([1e-3, -4e-4, 6e-4])       # eps11, eps22, gamma12
    Cs, angs = material.layer_material(cfg)
    # exact field: per layer, eps33 from sigma33 = 0 (out-of-plane shears decouple)
    zb = [0.0]
    e33 = []
    for li, L in enumerate(cfg["layers"]):
        Q = material.ply_axes(np.eye(3)[None], np.array([angs[li]]))[0]
        Cg = material.rotate_stiffness(Cs[li], Q)
        assert np.allclose(Cg[[0, 1, 2, 5]][:, [3, 4]], 0, atol=1e-8)
        e33.append(-(Cg[2, 0] * eps[0] + Cg[2, 1] * eps[1] + Cg[2, 5] * eps[2]) / Cg[2, 2])
        zb.append(zb[-1] + L["t"])
    x, y, z = mesh.xyz.T
    li = np.clip(np.searchsorted(zb, z, side="right") - 1, 0, len(angles) * 2 - 2)
    w = np.array([sum(e33[k] * cfg["layers"][k]["t"] for k in range(i)) for i in li])
    w = w + np.array(e33)[li] * (z - np.array(zb)[li])
    u = np.stack([eps[0] * x + 0.5 * eps[2] * y, 0.5 * eps[2] * x + eps[1] * y, w], 1).ravel()
    lat = mesh.lat
    lateral = ((lat[:, 0] == 0) | (lat[:, 0] == 2 * mesh.nx) | (lat[:, 1] == 0) |
               (lat[:, 1] == 2 * mesh.ny))
    fixed = np.repeat(lateral, 3)
    free = ~fixed
    Kff = K[free][:, free].tocsc()
    uf = spla.spsolve(Kff, -(K[free][:, fixed] @ u[fixed]))
    assert np.allclose(uf, u[free], rtol=1e-9, atol=1e-12)
    # strain energy equals the CLT membrane energy L W eps^T A eps / 2
    A = np.zeros((3, 3))
    for L in cfg["layers"]:
        if L["mat"] == "ply":
            from workloads import PLY
            A += L["t"] * clt_qbar(PLY["E1"], PLY["E2"], PLY["nu12"], PLY["G12"], L["angle"])
        else:
            from workloads import RESIN
            E_, nu = RESIN["E"], RESIN["nu"]
            A += L["t"] * clt_qbar(E_, E_, nu, E_ / (2 * (1 + nu)), 0.0)
    U_fe = 0.5 * u @ (K @ u)
    U_clt = 0.5 * cfg["length"] * cfg["width"] * eps @ A @ eps
    assert abs(U_fe - U_clt) <= 1e-11 * U_clt


def test_traction_resultant_cfg0():
    m = Mesh(workloads.cfg0())
    f = fem.load_vector(m).reshape(-1, 3)
    assert np.allclose(f.sum(0), [10.0 * 1.2, 0, 0], rtol=1e-13, atol=1e-13)
    assert np.all(f[m.lat[:, 0] != 2 * m.nx] == 0)


@pytest.mark.parametrize("amp", [0.0, 0.3])
def test_end_moment_resultants(amp):
    cfg = workloads.small_lsection(amp=amp)
    m = Mesh(cfg)
    f = fem.load_vector(m).reshape(-1, 3)
    T = total_thickness(cfg)
    assert np.abs(f.sum(0)).max() <= 1e-12 * np.abs(f).max()
    # limb 2 runs along -z; the moment about the y axis through the mid-thickness line
    end = m.lat[:, 0] == 2 * m.nx
    xm = cfg["limb"] + cfg["radius"] + 0.5 * T
    mom = np.sum((m.xyz[end, 0] - xm) * f[end, 2])
    assert abs(abs(mom) - cfg["load"]["M"] * cfg["width"]) <= 1e-10 * cfg["load"]["M"]

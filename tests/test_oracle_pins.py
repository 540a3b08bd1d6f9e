"""Pins of the oracle functions that the other oracle tests leave open: the wrinkle and the
L-section map (section 3, Eq. eq-wrinkle and the curved map after it), the local frame on
curved parts (section 2.1, read as the isoparametric-Jacobian frame), the through-thickness
stress functional and its modulus gradient, the overlap growth of the decomposition
(section 2.3), and the element count of the verification mesh (section 2.2).

Each check compares against something the mathematics fixes independently of the oracle's
own formulas: calculus, elementary geometry (circumcentres, chord lengths, mirror
symmetry), strain transformations built here from Q eps Q^T, homogeneity of linear
elasticity in the moduli, and brute-force lattice counts.
"""
import copy
import json
import math
import os

import numpy as np
import pytest

import workloads
from oracle import adjoint, dd, fem, material
from oracle.element import gauss_point_data, material_at_points
from oracle.mesh import Mesh, geometry_map, s_boundaries, total_thickness, wrinkle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---- wrinkle w(s) = A exp(-(s/L)^2) cos(2 pi s / L) -------------------------------------
def _lsec(amp=0.3, wlen=4.0, **k):
    return workloads.small_lsection(amp=amp, wlen=wlen, **k)


def test_wrinkle_special_values():
    cfg = _lsec()
    A, L = cfg["wrinkle"]
    s = np.array([0.0, L / 4, -L / 4, 3 * L / 4, L / 2, L])
    w = wrinkle(cfg, s)
    assert w[0] == A
    assert np.all(np.abs(w[1:4]) <= 4e-16 * A)              # cos zeros (rounding of pi)
    assert abs(w[4] + A * math.exp(-0.25)) <= 1e-15 * A     # cos(pi) = -1 at s = L/2
    assert abs(w[5] - A * math.exp(-1.0)) <= 1e-15 * A
    x = np.linspace(-3 * L, 3 * L, 101)
    assert np.array_equal(wrinkle(cfg, x), wrinkle(cfg, -x))   # even in s
    assert np.all(np.abs(wrinkle(cfg, x)) <= A * np.exp(-(x / L) ** 2) * (1 + 1e-15))
    flat = dict(cfg, geometry="flat", length=20.0)
    assert wrinkle(flat, np.array([10.0]))[0] == A            # centred at mid-length


def test_wrinkle_derivative_and_steepest_slope():
    """A five-point numerical derivative of the oracle's w(s) equals the product-rule
    derivative; the steepest slope at A = 0.3 mm, L_w = 4 mm is 24.11 degrees."""
    cfg = _lsec()
    A, L = cfg["wrinkle"]
    s = np.linspace(-2 * L, 2 * L, 4001)
    h = 1e-3
    num = (-wrinkle(cfg, s + 2 * h) + 8 * wrinkle(cfg, s + h) - 8 * wrinkle(cfg, s - h) +
           wrinkle(cfg, s - 2 * h)) / (12 * h)
    g = np.exp(-(s / L) ** 2)
    exact = A * g * (-2 * s / L ** 2 * np.cos(2 * np.pi * s / L) -
                     2 * np.pi / L * np.sin(2 * np.pi * s / L))
    assert np.abs(num - exact).max() <= 1e-9
    fine = np.linspace(-2 * L, 2 * L, 800001)
    d = (wrinkle(cfg, fine[1:]) - wrinkle(cfg, fine[:-1])) / (fine[1] - fine[0])
    slope = math.degrees(math.atan(np.abs(d).max()))
    assert abs(slope - 24.11) < 0.01, slope


# ---- L-section map --------------------------------------------------------------------
def _ends(cfg):
    T = total_thickness(cfg)
    rref = cfg["radius"] + 0.5 * T
    return -0.25 * math.pi * rref, 0.25 * math.pi * rref, rref, T


def _pt(cfg, s, zeta, l=0.0):
    s = np.atleast_1d(np.asarray(s, dtype=float))
    return geometry_map(cfg, s, np.full_like(s, l), np.full_like(s, zeta))


def test_lsection_arc_is_a_circle_about_the_limb_corner():
    """Without a wrinkle, three points of any through-thickness level on the arc have their
    circumcentre at (limb, 0) (x, z) and radius R + zeta."""
    cfg = _lsec(amp=0.0)
    sa, sb, rref, T = _ends(cfg)
    for zeta in (0.0, 0.3 * T, T):
        P = _pt(cfg, [sa + 0.1, 0.3, sb - 0.2], zeta)[:, [0, 2]]
        (ax, az), (bx, bz), (cx, cz) = P
        d = 2 * (ax * (bz - cz) + bx * (cz - az) + cx * (az - bz))
        ux = ((ax ** 2 + az ** 2) * (bz - cz) + (bx ** 2 + bz ** 2) * (cz - az) +
              (cx ** 2 + cz ** 2) * (az - bz)) / d
        uz = ((ax ** 2 + az ** 2) * (cx - bx) + (bx ** 2 + bz ** 2) * (ax - cx) +
              (cx ** 2 + cz ** 2) * (bx - ax)) / d
        assert abs(ux - cfg["limb"]) < 1e-11 and abs(uz) < 1e-11
        assert abs(math.hypot(ax - ux, az - uz) - (cfg["radius"] + zeta)) < 1e-11


def test_lsection_mid_surface_is_arc_length_parametrised_and_c1():
    """s is the mid-surface arc length: chord sums along the mid-surface give 2 limb +
    pi R_ref / 2 end to end and pi R_ref / 2 over the arc; the curve is C1 at both joins,
    limb 1 runs along +x and limb 2 along -z (a 90 degree corner)."""
    cfg = _lsec(amp=0.0)
    sa, sb, rref, T = _ends(cfg)
    limb = cfg["limb"]
    s = np.linspace(sa - limb, sb + limb, 200001)
    P = _pt(cfg, s, 0.5 * T)
    seg = np.linalg.norm(np.diff(P, axis=0), axis=1)
    assert abs(seg.sum() - (2 * limb + 0.5 * math.pi * rref)) < 1e-6
    Pa = _pt(cfg, np.linspace(sa, sb, 100001), 0.5 * T)
    arc = np.linalg.norm(np.diff(Pa, axis=0), axis=1).sum()
    assert abs(arc - 0.5 * math.pi * rref) < 1e-8
    h = 1e-7
    for sj, t_in in ((sa, (1, 0, 0)), (sb, (0, 0, -1))):
        left = (_pt(cfg, sj, 0.5 * T) - _pt(cfg, sj - h, 0.5 * T))[0] / h
        right = (_pt(cfg, sj + h, 0.5 * T) - _pt(cfg, sj, 0.5 * T))[0] / h
        assert np.abs(left - right).max() < 1e-6
        assert np.abs(left - np.array(t_in)).max() < 1e-6
    # the straight limbs: limb 1 horizontal at height R + zeta, limb 2 vertical
    z = _pt(cfg, np.linspace(sa - limb, sa, 7), 0.2)
    assert np.allclose(z[:, 2], cfg["radius"] + 0.2, atol=1e-14)
    v = _pt(cfg, np.linspace(sb, sb + limb, 7), 0.2)
    assert np.allclose(v[:, 0], cfg["limb"] + cfg["radius"] + 0.2, atol=1e-14)


def test_lsection_thickness_lines_are_normal_and_wrinkle_moves_along_them():
    """At fixed s the through-thickness segment is normal to the mid-surface and of length
    T; the wrinkle displaces every point by w(s) along that normal."""
    cfg0 = _lsec(amp=0.0)
    cfg = _lsec(amp=0.3)
    sa, sb, rref, T = _ends(cfg)
    for s in (sa - 1.0, sa + 0.7, 0.0, 0.9, sb + 0.5):
        tang = (_pt(cfg0, s + 1e-6, 0.5 * T) - _pt(cfg0, s - 1e-6, 0.5 * T))[0]
        tang /= np.linalg.norm(tang)
        nvec = (_pt(cfg0, s, T) - _pt(cfg0, s, 0.0))[0]
        assert abs(np.linalg.norm(nvec) - T) < 1e-12
        assert abs(tang @ nvec) < 1e-8
        shift = (_pt(cfg, s, 0.4) - _pt(cfg0, s, 0.4))[0]
        w = wrinkle(cfg, np.array([s]))[0]
        assert np.linalg.norm(shift - w * nvec / T) < 1e-12


# ---- local frame and material on curved parts -----------------------------------------
def _bond(Q):
    """6x6 T with eps_material = T eps_global (Voigt [11,22,33,23,13,12], engineering
    shears), built column by column from eps' = Q eps Q^T."""
    idx = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    T = np.zeros((6, 6))
    for J, (k, l) in enumerate(idx):
        e = np.zeros((3, 3))
        if k == l:
            e[k, k] = 1.0
        else:
            e[k, l] = e[l, k] = 0.5            # engineering shear 1 = tensor 1/2 + 1/2
        r = Q @ e @ Q.T
        for I, (i, j) in enumerate(idx):
            T[I, J] = r[i, j] if i == j else 2.0 * r[i, j]
    return T


def _ply_C(angle=0.0):
    cfg = dict(layers=[{"mat": "ply", "t": 1.0, "nel": 1, "angle": angle}])
    C, _ = material.layer_material(cfg)
    return C[0]


@pytest.mark.parametrize("angle", [0.0, 45.0])
def test_curved_frame_at_element_symmetry_plane(angle):
    """Gauss points at xi = 0 of an unwrinkled arc element lie on the element's mirror
    plane, so dx/dxi there is the circle's tangent at the element's mid-angle theta_m:
    the material stiffness must be C rotated about y by theta_m (and by the ply angle about
    the radial normal)."""
    layers = [{"mat": "ply", "t": 0.5, "nel": 2, "angle": angle}]
    cfg = _lsec(amp=0.0, nx=16, ny=2, layers=layers)
    mesh = Mesh(cfg)
    sa, sb, rref, T = _ends(cfg)
    sbd = s_boundaries(cfg)
    nl = cfg["nx_limb"]
    Cl = _ply_C(angle)
    checked = 0
    for ex in (nl, nl + 3, cfg["nx"] - nl - 1):
        e = ex                                  # (ez, ey) = (0, 0)
        X = mesh.xyz[mesh.conn[[e]]]
        gp = gauss_point_data(X)
        Cq = material_at_points(gp["J"], Cl[None], np.array([angle]))[0]
        th = (0.5 * (sbd[ex] + sbd[ex + 1]) - sa) / rref
        e1 = np.array([math.cos(th), 0.0, -math.sin(th)])
        e2 = np.array([0.0, 1.0, 0.0])
        e3 = np.cross(e1, e2)
        a = math.radians(angle)
        Q = np.stack([math.cos(a) * e1 + math.sin(a) * e2, -math.sin(a) * e1 + math.cos(a) * e2,
                      e3])
        Tb = _bond(Q)
        want = Tb.T @ Cl @ Tb
        for q in range(27):
            if q % 3 != 1:                      # xi = 0 points only
                continue
            assert np.abs(Cq[q] - want).max() <= 1e-9 * np.abs(want).max(), (ex, q)
            checked += 1
    assert checked == 27


# ---- the stress functional ------------------------------------------------------------
def _rot_y(phi):
    c, s = math.cos(phi), math.sin(phi)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


@pytest.mark.parametrize("mat", ["ply", "resin"])
def test_sigma33_of_uniform_strain_on_a_rotated_plate(mat):
    """A flat plate turned rigidly by 35 degrees about y: the laminate normal is
    e3 = R z everywhere.  For the uniform strain of a linear displacement field, sigma_33 =
    e3 . (C_g eps) e3 is uniform, with C_g = T^T C T (T the strain rotation to the material
    axes), and J = sigma_33^2 times the plate's volume."""
    layer = ({"mat": "ply", "t": 0.6, "nel": 2, "angle": 30.0} if mat == "ply" else
             {"mat": "resin", "t": 0.6, "nel": 2, "angle": 0.0})
    cfg = workloads.small_flat(nx=3, ny=2, layers=[layer], length=3.0, width=2.0)
    mesh = Mesh(cfg)
    R = _rot_y(math.radians(35.0))
    mesh.xyz = mesh.xyz @ R.T
    G = np.array([[2e-3, -1e-3, 5e-4], [3e-4, -1.5e-3, 2e-3], [-7e-4, 1e-3, 2.5e-3]])
    u = (mesh.xyz @ G.T).ravel()
    eps_t = 0.5 * (G + G.T)
    eps = np.array([eps_t[0, 0], eps_t[1, 1], eps_t[2, 2], 2 * eps_t[1, 2], 2 * eps_t[0, 2],
                    2 * eps_t[0, 1]])
    C, _ = material.layer_material(cfg)
    a = math.radians(layer["angle"])
    e1, e2, e3 = R[:, 0], R[:, 1], R[:, 2]
    Q = np.stack([math.cos(a) * e1 + math.sin(a) * e2, -math.sin(a) * e1 + math.cos(a) * e2, e3])
    Tb = _bond(Q)
    sig = Tb.T @ C[0] @ Tb @ eps
    S = np.array([[sig[0], sig[5], sig[4]], [sig[5], sig[1], sig[3]], [sig[4], sig[3], sig[2]]])
    s33 = e3 @ S @ e3
    J = adjoint.objective(mesh, u)
    vol = cfg["length"] * cfg["width"] * total_thickness(cfg)
    assert abs(J - s33 ** 2 * vol) <= 1e-11 * J
    # the wrong axes give clearly different values
    for wrong in (e1 @ S @ e1, e2 @ S @ e2, sig[2]):
        assert abs(wrong ** 2 * vol - J) > 1e-3 * J


def test_modulus_gradient_homogeneity_all_isotropic_laminate():
    """Linear elasticity with displacement BCs and traction loads: scaling every modulus by
    a common factor scales u by its inverse and leaves the stress unchanged, so J is
    homogeneous of degree 0 in the moduli and sum_k E_k dJ/dE_k = 0.  With only isotropic
    layers E_k is each layer's single modulus; the individual terms are far from zero."""
    layers = [{"mat": "resin", "t": 0.3, "nel": 1, "angle": 0.0, "E": 8.0e3},
              {"mat": "resin", "t": 0.2, "nel": 1, "angle": 0.0, "E": 12.0e3},
              {"mat": "resin", "t": 0.3, "nel": 1, "angle": 0.0, "E": 20.0e3}]
    cfg = workloads.small_lsection(nx=12, ny=2, layers=layers)
    R = adjoint.gradient(cfg)
    terms = np.array([L["E"] * R["dJdp"][2 + k] for k, L in enumerate(layers)])
    assert np.abs(terms).min() > 1e-3 * np.abs(terms).max()
    assert abs(terms.sum()) <= 1e-8 * np.abs(terms).max(), terms
    # one layer of one material: dJ/dE vanishes on its own
    one = workloads.small_lsection(nx=12, ny=2,
                                   layers=[{"mat": "resin", "t": 0.8, "nel": 2, "angle": 0.0}])
    R1 = adjoint.gradient(one)
    scale = abs(R1["J"]) / workloads.RESIN["E"]
    assert abs(R1["dJdp"][2]) <= 1e-8 * scale


# ---- overlap growth of the decomposition ----------------------------------------------
def _lattice_interior_count(x0, x1, y0, y1, nx, ny, nz):
    """Nodes (at most one odd lattice index) whose every element lies in the element box
    [x0, x1) x [y0, y1) x [0, nz): brute force over the doubled lattice."""
    cnt = 0
    for i2 in range(2 * nx + 1):
        for j2 in range(2 * ny + 1):
            for k2 in range(2 * nz + 1):
                if (i2 % 2) + (j2 % 2) + (k2 % 2) > 1:
                    continue
                # elements touching the node along x: those whose range contains i2 / 2
                ex = {i2 // 2} if i2 % 2 else {i2 // 2 - 1, i2 // 2}
                ey = {j2 // 2} if j2 % 2 else {j2 // 2 - 1, j2 // 2}
                ex = {e for e in ex if 0 <= e < nx}
                ey = {e for e in ey if 0 <= e < ny}
                if all(x0 <= e < x1 for e in ex) and all(y0 <= e < y1 for e in ey):
                    cnt += 1
    return cnt


@pytest.mark.parametrize("overlap", [1, 2])
def test_overlap_growth_is_box_growth(overlap):
    """Growing a box of elements `overlap` times by node adjacency adds `overlap` element
    layers on every side, corners included, clipped at the domain: (nx_j + 2o)(ny_j + 2o)nz
    elements for an inner box.  Interior nodes are the nodes of the grown box not on its
    cut faces."""
    layers = [{"mat": "ply", "t": 0.5, "nel": 2, "angle": 0.0}]
    cfg = workloads.small_flat(nx=9, ny=7, layers=layers, length=9.0, width=7.0)
    prob = fem.Problem(cfg)
    m = prob.mesh
    px, py = 3, 2
    part = dd.box_partition(m, px, py)
    dec = dd.Decomposition(prob, part, overlap)
    bx = [(p * m.nx) // px for p in range(px + 1)]
    by = [(p * m.ny) // py for p in range(py + 1)]
    for j in range(px * py):
        ix, iy = j % px, j // px
        x0, x1 = max(0, bx[ix] - overlap), min(m.nx, bx[ix + 1] + overlap)
        y0, y1 = max(0, by[iy] - overlap), min(m.ny, by[iy + 1] + overlap)
        assert len(dec.elems[j]) == (x1 - x0) * (y1 - y0) * m.nz, j
        ex, ey = m.eidx[dec.elems[j], 0], m.eidx[dec.elems[j], 1]
        assert ex.min() == x0 and ex.max() == x1 - 1 and ey.min() == y0 and ey.max() == y1 - 1
        assert len(dec.interior_nodes[j]) == _lattice_interior_count(x0, x1, y0, y1, m.nx,
                                                                     m.ny, m.nz), j


# ---- the verification mesh ------------------------------------------------------------
def test_verification_mesh_built_has_the_paper_element_count():
    """Section 2.2: the corner-unfolding model meshed with 56 elements along s and l and 6
    per ply and interface over 12 plies and 11 interfaces has 432,768 elements; built here
    as the L-section mesh (R = 6.6 mm, 3 mm limbs, W = 15 mm, 0.23 / 0.02 mm layers)."""
    g = json.load(open(os.path.join(GOLDEN, "paper_mesh_counts.json")))
    angles = [45, -45, 90, 0, -45, 45, -45, 45, 0, 90, 45, -45]
    layers = workloads.ply_layers(angles, 0.23, 6, 0.02, 6)
    cfg = dict(name="verification", geometry="lsection", radius=6.6, limb=3.0, width=15.0,
               nx=56, ny=56, nx_limb=workloads._limb_elems(56, 3.0, 6.6, layers),
               layers=layers, load={"kind": "moment", "M": workloads.PAPER_MOMENT})
    m = Mesh(cfg)
    assert m.n_elems == g["verification_elements"]
    assert abs(total_thickness(cfg) - g["verification_thickness_mm"]) < 1e-12
    assert m.nz == 23 * 6
    assert int(m.elayer.max()) == 22
    # every element has positive volume
    X = m.xyz[m.conn[:: 997]]
    assert np.all(gauss_point_data(X)["detJ"] > 0)

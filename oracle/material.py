"""Material stiffness of plies and resin interfaces (oracle; test infrastructure).

The model is 3-D linear elasticity with a general anisotropic stiffness tensor (section 2,
section 2.1) using the orthotropic ply and isotropic interface constants of Table 1.

Readings where the paper is silent:

* Voigt order [11, 22, 33, 23, 13, 12] with engineering shear strains; MPa and mm;
* compliance of an orthotropic solid in its material axes from (E_i, G_ij, nu_ij) with
  nu_ji / E_j = nu_ij / E_i, and C = S^-1;
* rotation of C is done here on the full fourth-order tensor,
  C'_ijkl = Q_pi Q_qj Q_rk Q_sl C_pqrs with Q_pi = a_p . e_i the direction cosines of the
  material axes a_p in the global basis e_i.
"""
from __future__ import annotations

import numpy as np

VOIGT = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]


def orthotropic_compliance(E1, E2, E3, G12, G13, G23, nu12, nu13, nu23):
    S = np.zeros((6, 6), dtype=np.result_type(E1, E2, E3, G12, G13, G23, nu12, nu13, nu23, 1.0))
    S[0, 0], S[1, 1], S[2, 2] = 1.0 / E1, 1.0 / E2, 1.0 / E3
    S[0, 1] = S[1, 0] = -nu12 / E1
    S[0, 2] = S[2, 0] = -nu13 / E1
    S[1, 2] = S[2, 1] = -nu23 / E2
    S[3, 3], S[4, 4], S[5, 5] = 1.0 / G23, 1.0 / G13, 1.0 / G12
    return S


def orthotropic_stiffness(**k):
    return np.linalg.inv(orthotropic_compliance(**k))


def isotropic_stiffness(E, nu):
    """Lame form: sigma = lambda tr(eps) I + 2 mu eps."""
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[0, 0] = C[1, 1] = C[2, 2] = lam + 2 * mu
    C[3, 3] = C[4, 4] = C[5, 5] = mu
    return C


def isotropic_as_engineering(E, nu):
    """Engineering constants of an isotropic solid, for use with orthotropic_stiffness."""
    G = E / (2 * (1 + nu))
    return dict(E1=E, E2=E, E3=E, G12=G, G13=G, G23=G, nu12=nu, nu13=nu, nu23=nu)


def voigt_to_tensor(C):
    T = np.zeros(C.shape[:-2] + (3, 3, 3, 3), dtype=C.dtype)
    for I, (i, j) in enumerate(VOIGT):
        for J, (k, l) in enumerate(VOIGT):
            v = C[..., I, J]
            for (a, b) in {(i, j), (j, i)}:
                for (c, d) in {(k, l), (l, k)}:
                    T[..., a, b, c, d] = v
    return T


def tensor_to_voigt(T):
    C = np.zeros(T.shape[:-4] + (6, 6), dtype=T.dtype)
    for I, (i, j) in enumerate(VOIGT):
        for J, (k, l) in enumerate(VOIGT):
            C[..., I, J] = T[..., i, j, k, l]
    return C


def rotate_stiffness(C, Q):
    """Stiffness C given in the material axes a_p (rows of Q, global components)."""
    T = voigt_to_tensor(C)
    R = np.einsum("...pi,...qj,...rk,...sl,...pqrs->...ijkl", Q, Q, Q, Q, T, optimize=True)
    return tensor_to_voigt(R)


def ply_axes(frame, angle_deg):
    """Material axes of a ply whose fibre is rotated by angle about the frame normal.

    frame[..., 0/1/2, :] are the unit vectors e1 (along s), e2 (along l), e3 (normal).
    Reading: fibre = cos(a) e1 + sin(a) e2, right-handed about e3.
    """
    a = np.deg2rad(angle_deg)[..., None]
    c, s = np.cos(a), np.sin(a)
    e1, e2, e3 = frame[..., 0, :], frame[..., 1, :], frame[..., 2, :]
    a1 = c * e1 + s * e2
    a2 = -s * e1 + c * e2
    return np.stack([a1, a2, e3], axis=-2)


def layer_material(cfg, engineering=False):
    """Per material layer: stiffness in its material axes (6x6) and ply angle."""
    from workloads import PLY, RESIN
    Cs, angs, eng = [], [], []
    for L in cfg["layers"]:
        if L["mat"] == "ply":
            k = dict(PLY)
            if "E1" in L:
                k["E1"] = L["E1"]
        else:
            k = isotropic_as_engineering(L.get("E", RESIN["E"]), RESIN["nu"])
        eng.append(k)
        Cs.append(orthotropic_stiffness(**k))
        angs.append(L["angle"])
    # extra materials after the layers: resin edge strips, then the stiff end column
    for key in ("edge_strip", "stiff_end"):
        if cfg.get(key):
            k = isotropic_as_engineering(cfg[key]["E"], cfg[key]["nu"])
            eng.append(k)
            Cs.append(orthotropic_stiffness(**k))
            angs.append(0.0)
    if engineering:
        return np.array(Cs), np.array(angs), eng
    return np.array(Cs), np.array(angs)

"""Pins of the oracle's material module (Table 1 constants, section 2.1 anisotropy).

Checked against facts fixed by elasticity: S C = I, the Lame form of isotropy, invariance
of a transversely isotropic solid under rotation about its axis, index swap under a 90
degree rotation, invariance of the Mandel-form spectrum, and the textbook plane-stress
reduced stiffness of classical lamination theory (written out independently below).
"""
import numpy as np
import pytest

from oracle import material as M
from workloads import PLY, RESIN

W = np.diag([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])


def rot_z(deg):
    a = np.deg2rad(deg)
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, s, 0], [-s, c, 0], [0, 0, 1.0]])


def test_compliance_inverse():
    S = M.orthotropic_compliance(**PLY)
    C = M.orthotropic_stiffness(**PLY)
    assert np.allclose(S @ C, np.eye(6), atol=1e-12)
    assert np.allclose(C, C.T, rtol=1e-13)
    assert np.all(np.linalg.eigvalsh(C) > 0)


def test_isotropic_matches_lame():
    C1 = M.orthotropic_stiffness(**M.isotropic_as_engineering(RESIN["E"], RESIN["nu"]))
    C2 = M.isotropic_stiffness(RESIN["E"], RESIN["nu"])
    assert np.allclose(C1, C2, rtol=1e-12)
    # isotropy: any rotation leaves C unchanged
    Q = np.linalg.qr(np.random.default_rng(1).standard_normal((3, 3)))[0]
    assert np.allclose(M.rotate_stiffness(C2, Q), C2, rtol=1e-12, atol=1e-9)


def test_ninety_degree_rotation_swaps_axes():
    C = M.orthotropic_stiffness(**PLY)
    Q = M.ply_axes(np.eye(3)[None], np.array([90.0]))[0]
    Cr = M.rotate_stiffness(C, Q)
    perm = [1, 0, 2, 4, 3, 5]          # 11<->22, 23<->13
    assert np.allclose(Cr, C[np.ix_(perm, perm)], atol=1e-9)


def test_transverse_isotropy_invariant_about_fibre():
    k = dict(PLY)
    k["G23"] = k["E2"] / (2 * (1 + k["nu23"]))
    C = M.orthotropic_stiffness(**k)
    a = np.deg2rad(37.0)
    Q = np.array([[1, 0, 0], [0, np.cos(a), np.sin(a)], [0, -np.sin(a), np.cos(a)]])
    assert np.allclose(M.rotate_stiffness(C, Q), C, rtol=1e-12, atol=1e-8)
    # ... but not for the Table 1 ply, whose G23 differs from E2 / (2 (1 + nu23))
    C0 = M.orthotropic_stiffness(**PLY)
    assert not np.allclose(M.rotate_stiffness(C0, Q), C0, rtol=1e-6)


def test_rotation_preserves_mandel_spectrum():
    C = M.orthotropic_stiffness(**PLY)
    Q = np.linalg.qr(np.random.default_rng(2).standard_normal((3, 3)))[0]
    if np.linalg.det(Q) < 0:
        Q[0] *= -1
    e0 = np.linalg.eigvalsh(W @ C @ W)
    e1 = np.linalg.eigvalsh(W @ M.rotate_stiffness(C, Q) @ W)
    assert np.allclose(e0, e1, rtol=1e-12)


def clt_qbar(E1, E2, nu12, G12, theta_deg):
    """Textbook plane-stress reduced stiffness rotated by theta (Jones, CLT)."""
    nu21 = nu12 * E2 / E1
    d = 1 - nu12 * nu21
    Q11, Q22, Q12, Q66 = E1 / d, E2 / d, nu12 * E2 / d, G12
    t = np.deg2rad(theta_deg)
    c, s = np.cos(t), np.sin(t)
    Qb = np.zeros((3, 3))
    Qb[0, 0] = Q11 * c**4 + 2 * (Q12 + 2 * Q66) * s**2 * c**2 + Q22 * s**4
    Qb[0, 1] = (Q11 + Q22 - 4 * Q66) * s**2 * c**2 + Q12 * (s**4 + c**4)
    Qb[1, 1] = Q11 * s**4 + 2 * (Q12 + 2 * Q66) * s**2 * c**2 + Q22 * c**4
    Qb[0, 2] = (Q11 - Q12 - 2 * Q66) * s * c**3 + (Q12 - Q22 + 2 * Q66) * s**3 * c
    Qb[1, 2] = (Q11 - Q12 - 2 * Q66) * s**3 * c + (Q12 - Q22 + 2 * Q66) * s * c**3
    Qb[2, 2] = (Q11 + Q22 - 2 * Q12 - 2 * Q66) * s**2 * c**2 + Q66 * (s**4 + c**4)
    Qb[1, 0], Qb[2, 0], Qb[2, 1] = Qb[0, 1], Qb[0, 2], Qb[1, 2]
    return Qb


def reduced_from_3d(Cg):
    """Condense sigma_33 = sigma_23 = sigma_13 = 0 out of the rotated 3-D stiffness."""
    ip, op = [0, 1, 5], [2, 3, 4]
    A = Cg[np.ix_(ip, ip)]
    B = Cg[np.ix_(ip, op)]
    D = Cg[np.ix_(op, op)]
    return A - B @ np.linalg.solve(D, B.T)


@pytest.mark.parametrize("theta", [0.0, 45.0, -45.0, 90.0, 30.0, -60.0])
def test_rotated_ply_matches_classical_lamination_theory(theta):
    C = M.orthotropic_stiffness(**PLY)
    Q = M.ply_axes(np.eye(3)[None], np.array([theta]))[0]
    Qb3 = reduced_from_3d(M.rotate_stiffness(C, Q))
    Qb2 = clt_qbar(PLY["E1"], PLY["E2"], PLY["nu12"], PLY["G12"], theta)
    assert np.allclose(Qb3, Qb2, rtol=1e-11, atol=1e-7)

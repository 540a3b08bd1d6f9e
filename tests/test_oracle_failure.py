"""Pins of the oracle's sech^2 defect (section 3, Eq. eq-f) and the delamination-onset
criterion (section 3.3, Eq. eq-Camanho).

* defect: d at its centre; its half-value distances along the arc, across the width and
  through the thickness, found by bisection on the oracle's own function, are the sech^2
  half-width asech(1/sqrt 2) times each direction's extent, and the inward one is twice the
  outward one (b2 = 1/2 inwards, 1/4 outwards); at the paper's extent pi b1 along s it is
  below 1e-2 d, as the paper states;
* steepest slope: the closed form 4 d / (3 sqrt 3 b1) (times 2 / r_def per unit arc length)
  against the largest numerical derivative of the oracle's defect along the arc;
* criterion: uniform stress states on a rigidly rotated resin plate (pure through-thickness
  tension, compression, and the two interlaminar shears) give F = sigma_r / 61, 0,
  tau / 97, in the rotated frame's axes; F is homogeneous of degree one in the load;
* the criterion only looks at the resin interface layers.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import failure, fem
from oracle.mesh import Mesh, defect, total_thickness

ASECH = math.acosh(math.sqrt(2.0))          # sech^2 x = 1/2 at x = asech(1/sqrt 2)


def _half_distance(fn, hi):
    lo = 0.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if fn(mid) > 0.5:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def test_defect_centre_half_widths_and_extent():
    cfg = workloads.defect_lsection(width=6.0)
    D = cfg["defect"]
    T = total_thickness(cfg)
    R = cfg["radius"]
    rref = R + 0.5 * T
    s0, l0, z0 = D["s_def"], D["l_def"], D["zeta_def"]
    f = lambda s, l, z: float(defect(cfg, np.array(s), np.array(l), np.array(z))) / D["d"]
    assert f(s0, l0, z0) == 1.0
    hs = _half_distance(lambda x: f(s0 + x, l0, z0), 10.0)
    hl = _half_distance(lambda x: f(s0, l0 + x, z0), 10.0)
    h_out = _half_distance(lambda x: f(s0, l0, z0 + x), 10.0)
    h_in = _half_distance(lambda x: f(s0, l0, z0 - x), 10.0)
    assert abs(hs - ASECH * D["b1"] * rref / 2) < 1e-12
    assert abs(hl - ASECH * cfg["width"] * D["b3"] / math.pi) < 1e-12
    assert abs(h_out - ASECH * R * D["b2_out"] / math.pi) < 1e-12
    assert abs(h_in / h_out - 2.0) < 1e-12
    # negligible (< 1e-2) at the paper's extent: pi b1 in its s, i.e. pi b1 R_ref / 2 here
    assert f(s0 + math.pi * D["b1"] * rref / 2, l0, z0) < 1e-2
    assert f(s0 - math.pi * D["b1"] * rref / 2, l0, z0) < 1e-2


@pytest.mark.parametrize("zeta_def", [None, 0.3])
def test_steepest_slope_closed_form(zeta_def):
    cfg = workloads.defect_lsection(d=0.4, zeta_def=zeta_def)
    D = cfg["defect"]
    T = total_thickness(cfg)
    R = cfg["radius"]
    rref = R + 0.5 * T
    rdef = R + D["zeta_def"]
    s = np.linspace(-3.0, 3.0, 600001)
    f = defect(cfg, s, np.full_like(s, D["l_def"]), np.full_like(s, D["zeta_def"]))
    # arc length at radius r_def: d(arc) = r_def d(theta) = (r_def / R_ref) ds
    dfds = np.diff(f) / (np.diff(s) * rdef / rref)
    brute = math.degrees(math.atan(np.abs(dfds).max()))
    closed = failure.steepest_slope_deg(D["d"], D["b1"], rdef)
    assert abs(brute - closed) < 1e-4, (brute, closed)
    assert abs(failure.amplitude_for_slope(closed, D["b1"], rdef) - D["d"]) < 1e-14


def _rotated_resin_plate():
    layer = {"mat": "resin", "t": 0.6, "nel": 2, "angle": 0.0}
    cfg = workloads.small_flat(nx=2, ny=2, layers=[layer], length=2.0, width=2.0)
    mesh = Mesh(cfg)
    c, s = math.cos(0.4), math.sin(0.4)
    Rm = np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]]) @ np.array(
        [[math.cos(0.3), -math.sin(0.3), 0], [math.sin(0.3), math.cos(0.3), 0], [0, 0, 1]])
    mesh.xyz = mesh.xyz @ Rm.T
    return cfg, mesh, Rm


def _u_for_local_stress(mesh, Rm, S_loc):
    """Displacement of the uniform strain whose isotropic stress is S_loc in the rotated
    frame (rows of Rm^T are that frame's axes in global components)."""
    E, nu = workloads.RESIN["E"], workloads.RESIN["nu"]
    S = Rm @ S_loc @ Rm.T                                   # global stress
    eps = ((1 + nu) * S - nu * np.trace(S) * np.eye(3)) / E  # isotropic compliance
    return (mesh.xyz @ eps.T).ravel()


@pytest.mark.parametrize("case", ["tension", "compression", "tau_rs", "tau_rl", "mixed"])
def test_camanho_on_uniform_stress_states(case):
    cfg, mesh, Rm = _rotated_resin_plate()
    S = np.zeros((3, 3))
    want = None
    if case == "tension":
        S[2, 2] = 30.5
        want = 0.5
    elif case == "compression":
        S[2, 2] = -50.0
        S[0, 0] = 20.0
        want = 0.0
    elif case == "tau_rs":
        S[0, 2] = S[2, 0] = 48.5
        want = 0.5
    elif case == "tau_rl":
        S[1, 2] = S[2, 1] = -97.0
        want = 1.0
    else:
        S[2, 2], S[0, 2], S[1, 2] = 61.0, 97.0, 97.0
        S[2, 0], S[2, 1] = 97.0, 97.0
        S[0, 0], S[1, 1], S[0, 1], S[1, 0] = 11.0, -7.0, 5.0, 5.0
        want = math.sqrt(3.0)
    u = _u_for_local_stress(mesh, Rm, S)
    R = failure.failure(mesh, u)
    loc = failure.local_stresses(mesh, u, np.arange(mesh.n_elems))
    # every Gauss point sees the prescribed local stress
    ref = np.array([S[0, 0], S[1, 1], S[2, 2], S[1, 2], S[0, 2], S[0, 1]])
    assert np.abs(loc - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
    assert abs(R["F_max"] - want) <= 1e-11
    F2 = failure.failure(mesh, 2.0 * u)["F_max"]
    assert abs(F2 - 2.0 * want) <= 1e-11
    assert failure.failure_moment(96.8, 2.0) == 48.4


def test_criterion_only_in_resin_interfaces_and_moment_scaling():
    cfg = workloads.defect_lsection(nx=16, ny=2, d=0.2, angles=(0, 90, 0))
    prob = fem.Problem(cfg)
    import scipy.sparse.linalg as spla
    u = prob.to_full(spla.spsolve(prob.K.tocsc(), prob.f))
    R = failure.failure(prob.mesh, u)
    resin = failure.interface_layers(cfg)
    assert list(resin) == [1, 3]
    assert R["layer"] in resin
    ply_el = ~np.isin(prob.mesh.elayer, resin)
    assert np.all(R["F_elem"][ply_el] == 0.0) and R["F_elem"].max() == R["F_max"]
    # the moment at initiation: F scales with the load
    R2 = failure.failure(prob.mesh, 3.0 * u)
    assert abs(R2["F_max"] - 3.0 * R["F_max"]) <= 1e-12 * R2["F_max"]
    assert R["interface_from_outer"] in (1, 2)

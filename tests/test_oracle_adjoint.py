"""Pins of the oracle's adjoint gradient of the through-thickness stress functional.

* the adjoint gradient (wrinkle amplitude and wavelength through the mesh, the modulus of
  plies and of a resin layer through the stiffness, partial derivatives by complex step)
  against a complex step through the whole problem - K(p + ih), f(p + ih) and a complex
  sparse solve, a forward sensitivity with no adjoint in it - and against central finite
  differences of J;
* dJ/du against a complex-step directional derivative of J;
* no wrinkle (A = 0): J does not depend on the wavelength, so dJ/dL_w = 0 exactly.
"""
import copy

import numpy as np
import pytest

import workloads
from oracle import adjoint


@pytest.fixture(scope="module")
def lsec():
    cfg = workloads.small_lsection(nx=12, ny=2)
    return cfg, adjoint.gradient(cfg)


def _perturbed(cfg, p, h):
    c = copy.deepcopy(cfg)
    A, Lw = c["wrinkle"]
    if p == 0:
        c["wrinkle"] = (A + h, Lw)
    elif p == 1:
        c["wrinkle"] = (A, Lw + h)
    else:
        L = c["layers"][p - 2]
        key = "E1" if L["mat"] == "ply" else "E"
        base = L.get(key, workloads.PLY["E1"] if L["mat"] == "ply" else workloads.RESIN["E"])
        L[key] = base + h
    return c


def _value(cfg, p):
    if p == 0:
        return cfg["wrinkle"][0]
    if p == 1:
        return cfg["wrinkle"][1]
    L = cfg["layers"][p - 2]
    return workloads.PLY["E1"] if L["mat"] == "ply" else workloads.RESIN["E"]


def _complex_step_total(cfg, p, h=1e-30):
    """dJ/dp by a complex step through the whole problem: K(p + ih), f(p + ih) and a
    complex sparse solve (forward sensitivity, exact to rounding; no adjoint involved)."""
    import scipy.sparse.linalg as spla
    from oracle.fem import Problem
    prob = Problem(_perturbed(cfg, p, 1j * h))
    u = prob.to_full(spla.spsolve(prob.K.tocsc(), prob.f))
    return adjoint.objective(prob.mesh, u).imag / h


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_adjoint_matches_complex_step_of_the_solve(lsec, p):
    cfg, R = lsec
    ref = _complex_step_total(cfg, p)
    # both routes solve with K (kappa ~ 1e8 here): they agree to about kappa * u
    assert abs(R["dJdp"][p] - ref) <= 1e-8 * abs(ref), (p, R["dJdp"][p], ref)


# FD steps (relative): J(p) carries the solves' rounding, about kappa(K) u ~ 1e-8 of J,
# which a step of 1e-6 |p| would amplify far beyond the 1e-5 target; these steps keep both
# that and the O(h^2) truncation below 1e-6
FD_REL = {0: 1e-4, 1: 1e-4, 2: 1e-3, 3: 1e-3, 4: 1e-3}


@pytest.mark.parametrize("p", [0, 2])
def test_adjoint_matches_central_differences(lsec, p):
    cfg, R = lsec
    h = FD_REL[p] * abs(_value(cfg, p))
    fd = (adjoint.objective_at(_perturbed(cfg, p, h)) -
          adjoint.objective_at(_perturbed(cfg, p, -h))) / (2 * h)
    assert abs(R["dJdp"][p] - fd) <= 1e-5 * abs(fd), (p, R["dJdp"][p], fd)


def test_objective_gradient_matches_complex_step(lsec):
    cfg, R = lsec
    mesh, u = R["prob"].mesh, R["u"]
    g = adjoint.objective_grad(mesh, u)
    v = np.random.default_rng(3).standard_normal(u.size)
    dj = adjoint.objective(mesh, u + 1j * 1e-30 * v).imag / 1e-30
    assert abs(g @ v - dj) <= 1e-10 * abs(dj)


def test_no_wrinkle_no_wavelength_sensitivity():
    cfg = workloads.small_lsection(nx=12, ny=2, amp=0.0)
    R = adjoint.gradient(cfg)
    assert R["dJdp"][1] == 0.0
    assert R["dJdp"][0] != 0.0

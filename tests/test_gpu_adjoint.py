"""GPU parity of the adjoint sensitivities of the through-thickness stress functional.

* J of the oracle's displacement: the library's objective kernel (strains rotated into the
  material axes) against the oracle's (global stress projected on the laminate normal),
  1e-12 relative;
* dJ/dp for the wrinkle amplitude and wavelength and every layer's modulus: the library's
  adjoint (dual-number element derivatives, PCG adjoint solve) against the oracle's
  (complex-step partial derivatives, direct solves).  Both use their own assembly of K,
  whose rounding differences (about 1e-14 of max |K|) move u and lambda by kappa(K) times
  that; with kappa ~ 1e8 on this L-section the bound is 1e-6 of the largest derivative;
* central finite differences of the library's own J(p), every solve on the GPU to
  rtol 1e-12, steps balanced between truncation and solve rounding: 1e-5 relative.
  (Steps of 1e-6 |p| would amplify the solves' rounding, about kappa(K) u ~ 1e-8 of J,
  to about 1e-2 of the derivative; 1e-4 |p| for the shape parameters and 1e-3 |p| for the
  moduli keep truncation and rounding both below 1e-6.)

Every primal and adjoint solve must converge (status GX_OK); none is taken from an
unconverged last iterate.
"""
import copy

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

FD_REL_SHAPE, FD_REL_MODULUS = 1e-4, 1e-3


def _fd_rel(p):
    return FD_REL_SHAPE if p < 2 else FD_REL_MODULUS


def _base(cfg, p):
    if p < 2:
        return cfg["wrinkle"][p]
    L = cfg["layers"][p - 2]
    return L.get("E1" if L["mat"] == "ply" else "E",
                 workloads.PLY["E1"] if L["mat"] == "ply" else workloads.RESIN["E"])


@pytest.fixture(scope="module")
def gx():
    import paper_1707_04228_amd as gx
    return gx


def _solve(gx, cfg, rtol=1e-12, x0=None):
    s = gx.Solver()
    s.laminate(cfg)
    f = s.assemble()
    sv = cfg["solver"]
    part = s.partition(cfg, sv["px"], sv["py"])
    s.geneo_setup(part, sv["px"] * sv["py"], overlap=sv["overlap"], tau=sv["tau"] or 0.1,
                  nev=sv["nev"] or 0, nev_max=sv["nev_max"])
    out = s.pcg(f, x=None if x0 is None else x0.clone(), rtol=rtol, maxit=3000)
    assert out["status"] == gx.GX_OK and out["relres"] <= rtol, (out["status"], out["relres"])
    return s, out["x"]


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
        L[key] = L.get(key, workloads.PLY["E1"] if L["mat"] == "ply" else workloads.RESIN["E"]) + h
    return c


@pytest.fixture(scope="module")
def lsec_oracle():
    from oracle import adjoint
    cfg = workloads.small_lsection(nx=12, ny=2)
    return cfg, adjoint.gradient(cfg)


def test_objective_matches_oracle(gx, lsec_oracle):
    import torch
    cfg, R = lsec_oracle
    s, _ = _solve(gx, cfg, rtol=1e-8)
    J = s.objective(torch.tensor(R["u"], device="cuda"), cfg)
    assert abs(J - R["J"]) <= 1e-12 * abs(R["J"])
    s.close()


def test_adjoint_matches_oracle(gx, lsec_oracle):
    cfg, R = lsec_oracle
    s, u = _solve(gx, cfg)
    J, g, it = s.adjoint(u, cfg, rtol=1e-12)
    ref = R["dJdp"]
    assert abs(J - R["J"]) <= 1e-6 * abs(R["J"])
    scale = np.abs(ref).max()
    assert np.all(np.abs(g - ref) <= 1e-6 * scale), (g, ref)
    # the derivatives that are not tiny agree to 1e-6 relative each
    big = np.abs(ref) > 1e-3 * scale
    assert np.all(np.abs(g - ref)[big] <= 1e-6 * np.abs(ref)[big])
    s.close()


@pytest.mark.parametrize("p", [0, 1, 2])
def test_gradient_matches_central_differences(gx, lsec_oracle, p):
    cfg, _ = lsec_oracle
    s, u = _solve(gx, cfg)
    _, g, _ = s.adjoint(u, cfg, rtol=1e-12)
    s.close()
    fd = _central_difference(gx, cfg, p)
    assert abs(g[p] - fd) <= 1e-5 * abs(fd), (p, g[p], fd)


def _central_difference(gx, cfg, p, rel=None, rtol=1e-12, x0=None):
    h = (rel or _fd_rel(p)) * abs(_base(cfg, p))
    Jp = []
    for sgn in (1, -1):
        c = _perturbed(cfg, p, sgn * h)
        sp, up = _solve(gx, c, rtol=rtol, x0=x0)
        Jp.append(sp.objective(up, c))
        sp.close()
    return (Jp[0] - Jp[1]) / (2 * h)


def _richardson_difference(gx, cfg, p, rel, rtol, x0):
    """(4 D(h) - D(2h)) / 3 of central differences D: truncation O(h^4), so a step large
    enough to drown the solves' rounding stays exact to far below 1e-5."""
    d1 = _central_difference(gx, cfg, p, rel, rtol, x0)
    d2 = _central_difference(gx, cfg, p, 2 * rel, rtol, x0)
    return (4 * d1 - d2) / 3


def test_no_wrinkle_no_wavelength_sensitivity(gx):
    cfg = workloads.small_lsection(nx=12, ny=2, amp=0.0)
    s, u = _solve(gx, cfg, rtol=1e-10)
    _, g, _ = s.adjoint(u, cfg, rtol=1e-10)
    assert g[1] == 0.0 and g[0] != 0.0
    s.close()


def test_autograd_function_returns_the_adjoint_gradient(gx, lsec_oracle):
    import torch
    cfg, R = lsec_oracle
    p = torch.tensor(gx.parameters_of(cfg), requires_grad=True)
    J = gx.laminate_objective(p, cfg)
    (2.0 * J).backward()
    ref = R["dJdp"]
    assert abs(J.item() - R["J"]) <= 1e-6 * abs(R["J"])
    assert np.all(np.abs(p.grad.numpy() - 2.0 * ref) <= 2e-6 * np.abs(ref).max())


def test_adjoint_at_full_size_matches_central_differences(gx):
    """The adjoint workload at its full size: the wrinkled L-section with 2 elements per
    ply, 240 x 4 x 35 elements (490,377 DOFs), 16 x 1 subdomains.  Too large for the
    oracle; checked by central differences of the library's own J (every solve on the GPU)
    for the wrinkle amplitude and wavelength, the 0 degree ply next to the inner radius and
    the off-axis ply (45, 90 or -45 degrees) whose E11 moves J most.  The off-axis moduli
    move J little (the 90 degree ply: dJ/dE11 ~ 7e-4, the 45 degree ply next to the inner
    radius ~ 1e-5, against 1.3e-2 for the 0 degree ply), and a central difference at
    1e-3 E11 carries about 2.5e-8 of noise from the solves (3e-10 of J); the plain central
    difference of L_w at 1e-4 L_w sits at the same noise level (a change of the mesh by one
    rounding moves it by 1e-5 relative).  Every parameter is therefore checked by a
    Richardson-extrapolated central difference (truncation O(h^4)) at 1e-3 |p| (1e-2 for
    the off-axis modulus) with solves to rtol 1e-13 started from u(p)."""
    cfg = workloads.cfg3()
    s, u = _solve(gx, cfg)
    assert 3 * s.mesh["n_nodes"] == 490377
    J, g, it = s.adjoint(u, cfg, rtol=1e-12)
    s.close()
    off = [2 + k for k, L in enumerate(cfg["layers"]) if L["mat"] == "ply" and L["angle"] != 0]
    p_off = max(off, key=lambda p: abs(g[p]))
    print(f"cfg3: off-axis ply with the largest dJ/dE11: layer {p_off - 2} "
          f"({cfg['layers'][p_off - 2]['angle']} deg), {g[p_off]:.4e}", flush=True)
    for p in (0, 1, 2, p_off):
        rel = 1e-2 if p == p_off else 1e-3
        fd = _richardson_difference(gx, cfg, p, rel, 1e-13, u)
        print(f"cfg3 p={p}: adjoint {g[p]:.10e} fd {fd:.10e}", flush=True)
        assert abs(g[p] - fd) <= 1e-5 * abs(fd), (p, g[p], fd)


def test_adjoint_is_bitwise_repeatable(gx):
    """dJ/du is gathered per node in a fixed order and every reduction has a fixed order, so
    two adjoint evaluations give the same J, iterations and dJ/dp bit for bit."""
    cfg = workloads.small_lsection(nx=12, ny=2)
    s, u = _solve(gx, cfg, rtol=1e-10)
    a = s.adjoint(u, cfg, rtol=1e-10)
    b = s.adjoint(u, cfg, rtol=1e-10)
    s.close()
    assert a[0] == b[0] and a[2] == b[2]
    assert np.array_equal(a[1], b[1])

"""GPU parity of the defect geometry and the delamination-onset criterion (section 3, Eq.
eq-f; section 3.3, Eq. eq-Camanho) against the oracle.

* the criterion kernel on the oracle's own displacement: F at every Gauss point within
  1e-10 of max F, the maximum and where it occurs equal (both FP64, same tie rule), the six
  local stresses there within 1e-9 of their largest;
* a layer mask that selects a ply instead of the interfaces gives the oracle's values for
  that ply;
* end to end (library mesh, assembly, GenEO PCG to rtol 1e-11, criterion) against the
  oracle's (direct solve): max F and the failure moment M / max F within 1e-7, the same
  element and point;
* deterministic: two evaluations agree bit for bit.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gx():
    import paper_1707_04228_amd as gx
    return gx


@pytest.fixture(scope="module")
def case():
    import scipy.sparse.linalg as spla
    from oracle import failure, fem
    cfg = workloads.defect_lsection(nx=20, ny=4, d=0.35)
    prob = fem.Problem(cfg)
    u = prob.to_full(spla.spsolve(prob.K.tocsc(), prob.f))
    return cfg, prob, u, failure.failure(prob.mesh, u)


def _oracle_gauss_F(prob, u, layers):
    from oracle import failure
    m = prob.mesh
    elems = np.nonzero(np.isin(m.elayer, layers))[0]
    loc = failure.local_stresses(m, u, elems)
    F = np.zeros((m.n_elems, 27))
    F[elems] = failure.camanho(loc)
    return F


def test_criterion_kernel_on_the_oracle_displacement(gx, case):
    import torch
    cfg, prob, u, R = case
    s = gx.Solver()
    s.laminate(cfg)
    s.assemble()
    ug = torch.tensor(u, device="cuda")
    out = s.failure(ug, per_gauss=True)
    Fg = out["F_gauss"].cpu().numpy().reshape(-1, 27)
    from oracle import failure
    Fo = _oracle_gauss_F(prob, u, failure.interface_layers(cfg))
    print(f"F_max gpu {out['F_max']:.15e} oracle {R['F_max']:.15e} at {out['elem']}/"
          f"{out['gauss']} vs {R['elem']}/{R['gauss']}", flush=True)
    assert np.abs(Fg - Fo).max() <= 1e-10 * R["F_max"]
    assert abs(out["F_max"] - R["F_max"]) <= 1e-10 * R["F_max"]
    assert (out["elem"], out["gauss"]) == (R["elem"], R["gauss"])
    assert out["layer"] == R["layer"]
    assert np.abs(out["stresses"] - R["stresses"]).max() <= 1e-9 * np.abs(R["stresses"]).max()
    assert np.array_equal(out["F_elem"].cpu().numpy(), Fg.max(axis=1))
    again = s.failure(ug)
    assert again["F_max"] == out["F_max"] and again["elem"] == out["elem"]
    assert torch.equal(again["F_elem"], out["F_elem"])
    # a ply selected instead of the interfaces
    ply = 2
    assert cfg["layers"][ply]["mat"] == "ply"
    op = s.failure(ug, layers=[ply])
    Rp = failure.failure(prob.mesh, u, layers=[ply])
    assert abs(op["F_max"] - Rp["F_max"]) <= 1e-10 * Rp["F_max"]
    assert op["layer"] == ply
    s.close()


def test_failure_end_to_end(gx, case):
    cfg, prob, u, R = case
    s = gx.Solver()
    s.laminate(cfg)
    f = s.assemble()
    sv = cfg["solver"]
    part = s.partition(cfg, sv["px"], sv["py"])
    s.geneo_setup(part, sv["px"] * sv["py"], overlap=sv["overlap"], nev=sv["nev"])
    sol = s.pcg(f, rtol=1e-11, maxit=1000)
    out = s.failure(sol["x"])
    M = cfg["load"]["M"]
    from oracle import failure
    print(f"end to end: F_max {out['F_max']:.12e} (oracle {R['F_max']:.12e}), failure moment "
          f"{failure.failure_moment(M, out['F_max']):.6f} N mm/mm", flush=True)
    assert abs(out["F_max"] - R["F_max"]) <= 1e-7 * R["F_max"]
    assert (out["elem"], out["gauss"]) == (R["elem"], R["gauss"])
    Mg, Mo = failure.failure_moment(M, out["F_max"]), failure.failure_moment(M, R["F_max"])
    assert abs(Mg - Mo) <= 1e-7 * Mo
    s.close()

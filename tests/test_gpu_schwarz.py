"""GPU parity of the overlapping decomposition, the one-level Schwarz preconditioner and
PCG against the oracle (section 2.3, Eq. eq-pre).

* partition: the library's box partition equals the oracle's (integer work, bit-exact);
* decomposition: per-subdomain interior DOF counts equal the oracle's (plus the clamped
  DOFs, which the library keeps as identity rows);
* P r: the one-level preconditioner applied by the library equals the oracle's (SuperLU
  subdomain solves) to 1e-9 relative, elementwise on the free DOFs;
* PCG: the same iteration count (+-1), residual histories within 1e-6 relative per
  iteration, and the solution within 1e-10 relative L2 of the oracle's at rtol 1e-8.
"""
import numpy as np
import pytest

import workloads
from gpu_helpers import rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gx():
    import paper_1707_04228_amd as gx
    return gx


def _setup(gx, cfg, coarse, precision=0, nev_per_sub=None):
    s = gx.Solver()
    s.laminate(cfg)
    f = s.assemble()
    sv = cfg["solver"]
    part = s.partition(cfg, sv["px"], sv["py"])
    s.geneo_setup(part, sv["px"] * sv["py"], overlap=sv["overlap"], tau=sv["tau"] or 0.1,
                  nev=sv["nev"] or 0, nev_max=sv["nev_max"], coarse=coarse,
                  precision=precision, nev_per_sub=nev_per_sub)
    return s, f, part


ONE_LEVEL = [workloads.cfg0(), workloads.small_lsection(nx=12, ny=2)]


@pytest.mark.parametrize("cfg", ONE_LEVEL, ids=lambda c: c["name"])
def test_one_level_preconditioner_and_pcg(gx, cfg):
    import torch
    from oracle import dd, fem, pcg
    s, f, part = _setup(gx, cfg, coarse=False)
    prob = fem.Problem(cfg)
    sv = cfg["solver"]
    opart = dd.box_partition(prob.mesh, sv["px"], sv["py"])
    assert np.array_equal(part.cpu().numpy(), opart)
    dec = dd.Decomposition(prob, opart, sv["overlap"])
    ni, nn, hb = s.subdomain_info()
    fixed = ~prob.free
    for j in range(dec.n_sub):
        nodes = dec.interior_nodes[j]
        n_fixed = int(fixed.reshape(-1, 3)[nodes].sum())
        assert ni[j] - n_fixed == len(dec.I[j])
    P = pcg.Schwarz(dec, None)
    rng = np.random.default_rng(11)
    r = rng.standard_normal(prob.n)
    r_full = torch.tensor(prob.to_full(r), device="cuda")
    z = s.precond(r_full).cpu().numpy()
    zo = P.apply(r)
    assert np.all(z[~prob.free] == 0)
    assert rel_err(z[prob.free], zo) <= 1e-9
    assert np.abs(z[prob.free] - zo).max() <= 1e-9 * np.abs(zo).max()
    # PCG trajectory
    out = s.pcg(f, rtol=1e-8, maxit=500, history=True)
    xo, ito, histo, _ = pcg.pcg(prob.K, prob.f, P.apply, rtol=1e-8)
    assert abs(out["iters"] - ito) <= 1
    k = min(len(out["hist"]), len(histo))
    assert np.all(np.abs(out["hist"][:k] - histo[:k]) <= 1e-6 * histo[:k])
    x = out["x"].cpu().numpy()
    assert np.all(x[~prob.free] == 0)
    assert rel_err(x[prob.free], xo) <= 1e-10

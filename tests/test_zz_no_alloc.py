"""The allocation-free objective (gx_objective_noalloc) against gx_objective and the oracle.

gx_objective_noalloc keeps its scratch in a static device array shared by every call on the
GPU.  Two calls in a row, the second on a smaller mesh, must each give gx_objective's J bit
for bit (same kernels, same summation order), and the oracle's J to 1e-12 relative (the two
assemblies' stresses differ by rounding only).
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def test_noalloc_objective_two_calls_shrinking():
    import torch
    import paper_1707_04228_amd as gx
    from oracle import adjoint, fem
    cases = [workloads.small_lsection(nx=24, ny=3), workloads.small_lsection(nx=12, ny=2)]
    solvers = []
    for k, cfg in enumerate(cases):
        s = gx.Solver()
        s.laminate(cfg)
        s.assemble()
        solvers.append(s)
        n = 3 * s.mesh["n_nodes"]
        rng = np.random.default_rng(100 + k)
        u_h = 1e-3 * rng.standard_normal(n)
        u = torch.tensor(u_h, device="cuda")
        prob = fem.Problem(cfg)
        u_o = u_h.copy()
        u_o[~prob.free] = 0.0
        u = torch.tensor(u_o, device="cuda")
        for region in (1, 0):
            J_ref = s.objective(u, region=region)
            J_na = s.objective_noalloc(u, region=region)
            print(f"case {cfg['name']} region {region}: J {J_ref:.17e} noalloc {J_na:.17e}",
                  flush=True)
            assert J_na == J_ref
        # the oracle's J on the arc (region 1)
        J_o = adjoint.objective(prob.mesh, u_o)
        assert abs(s.objective_noalloc(u, region=1) - J_o) <= 1e-12 * abs(J_o)
    for s in solvers:
        s.close()

"""Batched solves of several laminates (lockstep PCG over several contexts, one stream
each, per-laminate convergence).

* every laminate's solution and iteration count equal those of its own gx_pcg_solve on
  the same set-up: iteration counts within one and solutions within 1e-9 relative (the
  batch runs the same kernels per system, but the concurrent systems share the machine, so
  each band solve runs on fewer work-groups, which splits its sums differently: rounding);
* laminates of different size converge after different iteration counts and leave the
  batch independently;
* the work-group autotuner times its candidates and keeps the fastest; the solve after
  tuning still matches (to 1e-9 relative: a different work-group count splits the band
  solves differently, so the preconditioner changes by rounding and the two PCG runs to
  rtol 1e-10 drift apart by a few 1e-12; the iteration count stays within one).
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _cfgs():
    a = workloads.small_lsection(nx=12, ny=2)
    b = workloads.small_lsection(nx=12, ny=2, amp=0.1, wlen=6.0)
    c = workloads.cfg0()
    return [a, b, c]


def test_batch_matches_single_solves():
    import paper_1707_04228_amd as gx
    cfgs = _cfgs()
    batch = gx.Batch(cfgs)
    batch.setup()
    xs, it, rr, st = batch.solve(rtol=1e-10, maxit=500)
    assert np.all(st == gx.GX_OK)
    for k, cfg in enumerate(cfgs):
        s = batch.solvers[k]
        out = s.pcg(batch.f[k], rtol=1e-10, maxit=500)
        assert abs(out["iters"] - it[k]) <= 1
        assert rr[k] <= 1e-10
        x1, x2 = out["x"].cpu().numpy(), xs[k].cpu().numpy()
        assert np.abs(x1 - x2).max() <= 1e-9 * np.abs(x1).max()
    assert len(set(it.tolist())) > 1                # different convergence per laminate
    batch.close()


def test_autotune_keeps_the_fastest_and_the_solution():
    import paper_1707_04228_amd as gx
    cfg = workloads.cfg0()
    batch = gx.Batch([cfg])
    batch.setup()
    s = batch.solvers[0]
    o1 = s.pcg(batch.f[0], rtol=1e-10, maxit=500)
    ref = o1["x"].cpu().numpy()
    times = s.autotune(candidates=(1, 2, 3))
    assert set(times) == {1, 2, 3} and all(t > 0 for t in times.values())
    o2 = s.pcg(batch.f[0], rtol=1e-10, maxit=500)
    x = o2["x"].cpu().numpy()
    assert abs(o2["iters"] - o1["iters"]) <= 1
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()
    batch.close()

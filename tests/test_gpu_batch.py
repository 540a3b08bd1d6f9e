"""Batched solves of several laminates (lockstep PCG over several contexts, one stream
each, per-laminate convergence).

* every laminate's solution and iteration count equal those of its own gx_pcg_solve on
  the same set-up, in FP64 and with FP32 factors: iteration counts within one and solutions
  within 1e-9 relative (the batch runs the subdomain solves of all systems in one launch,
  whose work-group count per matrix differs from the lone solve's, so the band sums are
  split differently: rounding);
* a context listed twice is refused (GX_EINVAL);
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


def test_batch_fp32_factors_match_single_solves():
    import paper_1707_04228_amd as gx
    cfgs = _cfgs()
    batch = gx.Batch(cfgs, precision=gx.GX_MIXED)
    batch.setup()
    xs, it, rr, st = batch.solve(rtol=1e-10, maxit=500)
    assert np.all(st == gx.GX_OK)
    for k in range(len(cfgs)):
        out = batch.solvers[k].pcg(batch.f[k], rtol=1e-10, maxit=500)
        assert abs(out["iters"] - it[k]) <= 1
        assert rr[k] <= 1e-10
        x1, x2 = out["x"].cpu().numpy(), xs[k].cpu().numpy()
        assert np.abs(x1 - x2).max() <= 1e-9 * np.abs(x1).max()
    batch.close()


def test_batch_refuses_a_context_twice():
    import ctypes as C
    import torch
    import paper_1707_04228_amd as gx
    batch = gx.Batch([workloads.cfg0()])
    batch.setup()
    s, f = batch.solvers[0], batch.f[0]
    x = torch.zeros_like(f)
    vp = C.c_void_p
    H = (vp * 2)(s.h, s.h)
    Bp = (vp * 2)(f.data_ptr(), f.data_ptr())
    Xp = (vp * 2)(x.data_ptr(), x.data_ptr())
    it = np.zeros(2, dtype=np.int32)
    rr = np.zeros(2)
    st = np.zeros(2, dtype=np.int32)
    code = gx.lib.gx_pcg_solve_batch(2, H, Bp, Xp, 1e-8, 100,
                                     it.ctypes.data_as(C.POINTER(C.c_int32)),
                                     rr.ctypes.data_as(C.POINTER(C.c_double)),
                                     st.ctypes.data_as(C.POINTER(C.c_int32)))
    assert code == gx.GX_EINVAL
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

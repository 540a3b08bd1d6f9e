"""Batched solves of several laminates (lockstep PCG over several contexts, one stream
each, per-laminate convergence).

* every laminate's solution and iteration count equal those of its own gx_pcg_solve on
  the same set-up, in FP64 and with FP32 factors: iteration counts within one and solutions
  within 1e-9 relative (the batch runs the subdomain solves of all systems in one launch,
  whose work-group count per matrix differs from the lone solve's, so the band sums are
  split differently: rounding);
* a context listed twice is refused (GX_EINVAL);
* set-ups run concurrently (gx_geneo_setup_batch, three at a time) keep the modes and
  eigenvalues of one-at-a-time set-ups (eigenvalues within 1e-8 relative: the concurrent
  eigensolver block solves run on fewer work-groups, which changes rounding only), and
  the PCG on them takes the same iterations (within one) to the same solution; a set-up
  that fails is reported for its own laminate while the others complete;
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


def test_concurrent_setup_matches_one_at_a_time():
    import paper_1707_04228_amd as gx
    cfgs = _cfgs()
    b1 = gx.Batch(cfgs)
    r1 = b1.setup(concurrent=1)
    b3 = gx.Batch(cfgs)
    r3 = b3.setup(concurrent=3)
    for k in range(len(cfgs)):
        assert np.array_equal(r1[k][0], r3[k][0]) and r1[k][1] == r3[k][1]
        for j in range(len(r1[k][0])):
            l1 = b1.solvers[k].eigenvalues(j)
            l3 = b3.solvers[k].eigenvalues(j)
            assert np.abs(l1 - l3).max() <= 1e-8 * np.abs(l1).max()
    x1, i1, _, s1 = b1.solve(rtol=1e-10, maxit=500)
    x3, i3, _, s3 = b3.solve(rtol=1e-10, maxit=500)
    assert np.all(s1 == gx.GX_OK) and np.all(s3 == gx.GX_OK)
    assert np.all(np.abs(i1 - i3) <= 1)
    for a, b in zip(x1, x3):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.abs(a - b).max() <= 1e-9 * np.abs(a).max()
    b1.close()
    b3.close()


def test_concurrent_setup_reports_a_failure_per_laminate():
    import ctypes as C
    import paper_1707_04228_amd as gx
    cfgs = _cfgs()[:2]
    batch = gx.Batch(cfgs)
    parts, opts = [], []
    for cfg, s in zip(cfgs, batch.solvers):
        sv = cfg["solver"]
        part = s.partition(cfg, sv["px"], sv["py"])
        parts.append(part)
        opts.append(gx.GeneoOpts(sv["px"] * sv["py"], part.data_ptr(), sv["overlap"], 0.1, 0,
                                 32, gx.GX_FP64, 1, None, 0.0, 0))
    opts[1].overlap = 0                             # invalid: refused by that set-up alone
    vp = C.c_void_p
    H = (vp * 2)(*[s.h for s in batch.solvers])
    O = (C.POINTER(gx.GeneoOpts) * 2)(*[C.pointer(o) for o in opts])
    st = np.full(2, -1, dtype=np.int32)
    n0 = np.zeros(2, dtype=np.int64)
    code = gx.lib.gx_geneo_setup_batch(2, H, O, 2, None, n0.ctypes.data_as(C.POINTER(C.c_int64)),
                                       st.ctypes.data_as(C.POINTER(C.c_int32)))
    assert code == gx.GX_EINVAL
    assert st[0] == gx.GX_OK and st[1] == gx.GX_EINVAL and n0[0] > 0
    assert "overlap" in gx.lib.gx_last_error(batch.solvers[1].h).decode()
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


def test_batch_of_seeded_samples_matches_the_oracle():
    """Two laminates drawn from the seeded wrinkle-sample sweep (different ply counts,
    amplitudes and wavelengths; meshes reduced to 16 x 2 elements in plane) solved together
    by the batched PCG with FP32 factors, each against the oracle's exact solution of its own
    system (refined sparse LU): within 1e-8 at rtol 1e-10."""
    import paper_1707_04228_amd as gx
    from oracle import fem
    from test_gpu_schwarz import refined_solve
    smp = workloads.cfg4_samples()
    picks = [0, next(i for i in range(1, 32) if len(smp[i]["angles"]) != len(smp[0]["angles"]))]
    cfgs = []
    for i in picks:
        layers = workloads.ply_layers(smp[i]["angles"], 0.25, 1, 0.05, 1)
        c = workloads.small_lsection(nx=16, ny=2, amp=smp[i]["amp"], wlen=smp[i]["wlen"],
                                     layers=layers)
        c["name"] = f"sample{i}_16x2"
        cfgs.append(c)
    batch = gx.Batch(cfgs, precision=gx.GX_MIXED)
    batch.setup()
    xs, it, rr, st = batch.solve(rtol=1e-10, maxit=1000)
    assert np.all(st == gx.GX_OK)
    for k, cfg in enumerate(cfgs):
        prob = fem.Problem(cfg)
        xo, _ = refined_solve(prob.K, prob.f)
        x = xs[k].cpu().numpy()[prob.free]
        err = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        print(f"{cfg['name']} ({len(cfg['layers'])} layers): {it[k]} iterations, error vs the "
              f"oracle {err:.2e}", flush=True)
        assert err <= 1e-8
    batch.close()

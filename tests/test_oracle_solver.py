"""Pins of the oracle's decomposition, GenEO coarse space and PCG (section 2.3, Eq. eq-pre).

* PCG at a tight tolerance reproduces a direct sparse solve of K u = f;
* one subdomain covering the mesh makes P = K^-1, so CG stops after one iteration;
* the partition of unity sums to the identity on the free DOFs;
* P is symmetric and positive definite, K_0 is SPD;
* on floating subdomains the six smallest GenEO eigenvalues vanish and their eigenvectors
  are the local rigid-body modes (section 2.3, Fig. fig-eig);
* ARPACK shift-invert agrees with a dense generalised eigensolve on small subdomains.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import dd, fem, geneo, pcg


@pytest.fixture(scope="module")
def small():
    cfg = workloads.small_flat(nx=6, ny=4)
    cfg["solver"].update(px=3, py=2, overlap=1, nev=6)
    return pcg.solve(cfg, rtol=1e-12)


def test_pcg_matches_direct_solve(small):
    prob = small["prob"]
    xd = spla.spsolve(prob.K.tocsc(), prob.f)
    assert np.linalg.norm(small["x"] - xd) <= 1e-10 * np.linalg.norm(xd)


def test_cfg0_pcg_matches_direct(cfg0_oracle):
    prob = cfg0_oracle["prob"]
    xd = spla.spsolve(prob.K.tocsc(), prob.f)
    x, it, hist, _ = pcg.pcg(prob.K, prob.f, cfg0_oracle["P"].apply, rtol=1e-12)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    assert it < 60


def test_coarse_space_keeps_iterations_bounded():
    """Section 2.4: one-level Schwarz iterations grow with the number of subdomains while
    the GenEO two-level method stays far lower (qualitative; the paper's counts are for
    another model)."""
    its = {}
    for px in (4, 8):
        cfg = workloads.small_flat(nx=4 * px, ny=2, length=4.0 * px, width=2.0)
        cfg["solver"].update(px=px, py=1, overlap=1, nev=0, tau=0.1)
        its[px] = (pcg.solve(cfg, rtol=1e-10)["iters"],
                   pcg.solve(cfg, rtol=1e-10, one_level=True)["iters"])
    assert its[8][1] > 2 * its[4][1] * 0.9          # one-level roughly doubles
    assert its[8][0] < 1.6 * its[4][0]              # two-level grows much less
    assert its[8][0] < 0.5 * its[8][1]


def test_single_subdomain_is_exact():
    cfg = workloads.small_flat(nx=3, ny=2)
    prob = fem.Problem(cfg)
    part = np.zeros(prob.mesh.n_elems, dtype=np.int64)
    dec = dd.Decomposition(prob, part, 1)
    assert len(dec.I[0]) == prob.n
    P = pcg.Schwarz(dec, None)
    x, it, hist, _ = pcg.pcg(prob.K, prob.f, P.apply, rtol=1e-10)
    assert it == 1


def test_partition_of_unity(small):
    dec = small["dec"]
    s = np.zeros(dec.prob.n)
    for Ij, Xj in zip(dec.I, dec.X):
        s[Ij] += Xj
    assert np.allclose(s, 1.0, atol=1e-15)
    # every subdomain interior lies inside its Neumann DOF set
    for Ij, Dj in zip(dec.I, dec.D):
        assert np.all(np.isin(Ij, Dj))


def test_preconditioner_symmetric_positive(small):
    rng = np.random.default_rng(3)
    n = small["prob"].n
    P = small["P"].apply
    for _ in range(3):
        x, y = rng.standard_normal(n), rng.standard_normal(n)
        a, b = x @ P(y), y @ P(x)
        assert abs(a - b) <= 1e-12 * (abs(a) + abs(b) + np.linalg.norm(x) * np.linalg.norm(P(x)))
        assert x @ P(x) > 0
    K0 = small["coarse"].K0
    assert np.allclose(K0, K0.T)
    assert np.linalg.eigvalsh(K0)[0] > 0


def test_floating_subdomain_rigid_modes(cfg0_oracle):
    dec, coarse = cfg0_oracle["dec"], cfg0_oracle["coarse"]
    mesh = dec.prob.mesh
    touches_clamp = [np.any(mesh.lat[dec.touch_nodes[j], 0] == 0) for j in range(dec.n_sub)]
    assert any(touches_clamp) and not all(touches_clamp)
    for j in range(dec.n_sub):
        lam = coarse.lams[j]
        if touches_clamp[j]:
            assert lam[0] > 1e-6
            continue
        assert np.all(np.abs(lam) < 1e-9)
        AN, B, xt, pos = geneo.local_matrices(dec, j)
        _, V = geneo.solve_local_eigen(AN, B, nev=6)
        # eigenvectors span the rigid-body modes of the subdomain's nodes
        nodes = dec.touch_nodes[j]
        xyz = mesh.xyz[nodes]
        R = []
        for c in range(3):
            t = np.zeros_like(xyz)
            t[:, c] = 1
            R.append(t.ravel())
        for ax in np.eye(3):
            R.append(np.cross(ax, xyz).ravel())
        R = np.array(R).T
        Q, _ = np.linalg.qr(V)
        assert np.linalg.norm(R - Q @ (Q.T @ R)) <= 1e-8 * np.linalg.norm(R)


def test_arpack_matches_dense_eigen(small):
    dec = small["dec"]
    for j in range(dec.n_sub):
        AN, B, xt, pos = geneo.local_matrices(dec, j)
        l1, V1 = geneo.solve_local_eigen(AN, B, nev=8, dense=False)
        l2, V2 = geneo.solve_local_eigen(AN, B, nev=8, dense=True)
        assert np.allclose(l1, l2, atol=1e-9, rtol=1e-8)
        # eigen-residuals of the pencil
        r = AN @ V1 - (B @ V1) * l1[None, :]
        assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(AN @ V1)


def test_threshold_selection():
    cfg = workloads.small_flat(nx=6, ny=4)
    cfg["solver"].update(px=3, py=2, overlap=1, nev=0, tau=0.1)
    R = pcg.solve(cfg, rtol=1e-10)
    for lam in R["coarse"].lams:
        assert np.all(lam < 0.1)
    assert R["iters"] < 60


def test_arpack_clustered_spectrum_and_cap():
    """tau = 1.2 on the small L-section: about 30 eigenvalues per subdomain below the
    threshold, clustered near 1, and the cap nev_max = 32 binding in the middle subdomain.
    The sparse path equals the dense generalised eigensolver (eigenvalues, and the span of
    the selected vectors), also after unrelated ARPACK calls: the start vector is fixed and
    the returned block is purified."""
    cfg = workloads.small_lsection(nx=12, ny=2)
    prob = fem.Problem(cfg)
    sv = cfg["solver"]
    dec = dd.Decomposition(prob, dd.box_partition(prob.mesh, sv["px"], sv["py"]),
                           sv["overlap"])
    counts = []
    for j in range(dec.n_sub):
        AN, B, xt, pos = geneo.local_matrices(dec, j)
        l2, V2 = geneo.solve_local_eigen(AN, B, tau=1.2, nev_max=32, dense=True)
        for _ in range(2):                         # the second run follows other calls
            spla.eigsh(AN, k=3, which="LM", return_eigenvectors=False)
            l1, V1 = geneo.solve_local_eigen(AN, B, tau=1.2, nev_max=32, dense=False)
            assert len(l1) == len(l2)
            assert np.all(np.abs(l1 - l2) <= 1e-10 * np.abs(l2) + 1e-10)   # zero modes: noise
            Q1, _ = np.linalg.qr(V1)
            Q2, _ = np.linalg.qr(V2)
            s = np.linalg.svd(Q1.T @ Q2, compute_uv=False)
            assert s.min() >= 1 - 1e-12                # principal angles below ~1.4e-6
        counts.append(len(l1))
    assert max(counts) == 32 and min(counts) > 24

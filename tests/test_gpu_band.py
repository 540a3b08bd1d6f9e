"""GPU parity of the subdomain solver in isolation: batched banded Cholesky factorisation
and triangular solves (section 2.4, exact local solves), against SciPy's banded Cholesky
(LAPACK pbtrf/pbtrs) on the same matrices.

Shapes cover a single 64-row block, ragged tails, bandwidths below, at and above the block
size, a bandwidth of n - 1 (dense), and the orders and bandwidths of the subdomain and
eigensolver matrices of the small test laminates; every right-hand-side count the solver
takes (1, 8, 16, 24, 32) and several work-group counts per matrix (the pipelined sweeps).
FP64: componentwise within 1e-10 of the LAPACK solution relative to its largest entry
(both are backward-stable solves of well-conditioned matrices, kappa < 1e3 here).  Mixed
precision (FP32 factors of the equilibrated matrix): within 1e-4.
"""
import numpy as np
import pytest
import scipy.linalg as sla

pytestmark = pytest.mark.gpu

SHAPES = [(64, 10), (65, 3), (1, 0), (130, 129), (200, 70), (257, 64), (300, 299),
          (945, 218), (1269, 290), (1080, 248), (4395, 398)]


@pytest.fixture(scope="module")
def solver():
    import paper_1707_04228_amd as gx
    s = gx.Solver()
    yield gx, s
    s.close()


def _band_spd(n, B, rng):
    """Random SPD band matrix (diagonally dominant) in row-major band storage and as the
    LAPACK lower band form."""
    lo = np.zeros((B + 1, n))                      # lo[d, c] = A[c + d, c]
    for d in range(1, B + 1):
        lo[d, : n - d] = rng.uniform(-1.0, 1.0, n - d)
    rowsum = np.zeros(n)
    for d in range(1, B + 1):
        rowsum[: n - d] += np.abs(lo[d, : n - d])
        rowsum[d:] += np.abs(lo[d, : n - d])
    lo[0] = rowsum + rng.uniform(1.0, 2.0, n)
    band = np.zeros(n * (B + 1))
    for d in range(B + 1):                        # entry (r, r - d) at r (B + 1) + B - d
        r = np.arange(d, n)
        band[r * (B + 1) + B - d] = lo[d, : n - d]
    return band, lo


@pytest.mark.parametrize("nrhs", [1, 8, 16, 24, 32, 40, 48])
@pytest.mark.parametrize("groups", [0, 1, 3])
def test_band_factor_solve_fp64(solver, nrhs, groups):
    import torch
    gx, s = solver
    rng = np.random.default_rng(100 + nrhs + 7 * groups)
    bands, los, xs = [], [], []
    for n, B in SHAPES:
        band, lo = _band_spd(n, B, rng)
        bands.append(band)
        los.append(lo)
        xs.append(rng.standard_normal((n, nrhs)))
    band_t = torch.tensor(np.concatenate(bands), device="cuda")
    x_t = torch.tensor(np.concatenate([x.ravel() for x in xs]), device="cuda")
    s.band_factor_solve([n for n, _ in SHAPES], [B for _, B in SHAPES], band_t, x_t,
                        precision=gx.GX_FP64, groups=groups)
    got = x_t.cpu().numpy()
    o = 0
    for (n, B), lo, x in zip(SHAPES, los, xs):
        ref = sla.cho_solve_banded((sla.cholesky_banded(lo, lower=True), True), x)
        g = got[o: o + n * nrhs].reshape(n, nrhs)
        o += n * nrhs
        assert np.abs(g - ref).max() <= 1e-10 * np.abs(ref).max(), (n, B)


@pytest.mark.parametrize("nrhs", [1, 16, 48])
def test_band_factor_solve_mixed(solver, nrhs):
    import torch
    gx, s = solver
    rng = np.random.default_rng(7 + nrhs)
    bands, los, xs = [], [], []
    for n, B in SHAPES:
        band, lo = _band_spd(n, B, rng)
        bands.append(band)
        los.append(lo)
        xs.append(rng.standard_normal((n, nrhs)))
    band_t = torch.tensor(np.concatenate(bands), device="cuda")
    x_t = torch.tensor(np.concatenate([x.ravel() for x in xs]), device="cuda")
    s.band_factor_solve([n for n, _ in SHAPES], [B for _, B in SHAPES], band_t, x_t,
                        precision=gx.GX_MIXED)
    got = x_t.cpu().numpy()
    o = 0
    for (n, B), lo, x in zip(SHAPES, los, xs):
        ref = sla.cho_solve_banded((sla.cholesky_banded(lo, lower=True), True), x)
        g = got[o: o + n * nrhs].reshape(n, nrhs)
        o += n * nrhs
        assert np.abs(g - ref).max() <= 1e-4 * np.abs(ref).max(), (n, B)


# launches whose widest matrix has fewer 64-row blocks below a panel than a factorisation
# group has panels (the group's own rows are then the whole band, or nearly), and one with
# no off-diagonal entries at all
NARROW = [[(300, 50), (129, 10), (64, 63), (700, 63)],
          [(513, 127), (300, 120), (1, 0), (1000, 100)],
          [(5, 0), (300, 0), (257, 0)]]


@pytest.mark.parametrize("shapes", NARROW)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("nrhs", [1, 16])
def test_band_factor_solve_narrow_bands(solver, shapes, precision, nrhs):
    import torch
    gx, s = solver
    rng = np.random.default_rng(11 + nrhs + len(shapes))
    bands, los, xs = [], [], []
    for n, B in shapes:
        band, lo = _band_spd(n, B, rng)
        bands.append(band)
        los.append(lo)
        xs.append(rng.standard_normal((n, nrhs)))
    band_t = torch.tensor(np.concatenate(bands), device="cuda")
    x_t = torch.tensor(np.concatenate([x.ravel() for x in xs]), device="cuda")
    prec = gx.GX_FP64 if precision == "fp64" else gx.GX_MIXED
    s.band_factor_solve([n for n, _ in shapes], [B for _, B in shapes], band_t, x_t,
                        precision=prec)
    got = x_t.cpu().numpy()
    tol = 1e-10 if precision == "fp64" else 1e-4
    o = 0
    for (n, B), lo, x in zip(shapes, los, xs):
        ref = sla.cho_solve_banded((sla.cholesky_banded(lo, lower=True), True), x)
        g = got[o: o + n * nrhs].reshape(n, nrhs)
        o += n * nrhs
        assert np.abs(g - ref).max() <= tol * np.abs(ref).max(), (n, B)


def test_band_rejects_bad_input(solver):
    import torch
    gx, s = solver
    band = torch.zeros(10, dtype=torch.float64, device="cuda")
    x = torch.zeros(5 * 3, dtype=torch.float64, device="cuda")
    with pytest.raises(gx.GxError):                # 3 right-hand sides: not supported
        s.band_factor_solve([5], [1], band, x)
    x = torch.zeros(5 * 72, dtype=torch.float64, device="cuda")
    with pytest.raises(gx.GxError):                # 72: more than 64 not supported
        s.band_factor_solve([5], [1], band, x)
    x = torch.zeros(5, dtype=torch.float64, device="cuda")
    with pytest.raises(gx.GxError):                # zero matrix: not positive definite
        s.band_factor_solve([5], [1], band, x)

"""Host-side bounds check of the band kernels' unconditional loads.

The band solves and the trailing update issue their loads unconditionally from clamped
addresses and apply the band mask afterwards (so a wave issues every load of a step before
it waits for any).  Such a load may read outside the band, and past the last row of the
last matrix: the band allocation carries BAND_PAD trailing entries for that.  This test
restates every clamped address expression of those kernels (paper_1707_04228_amd/csrc/
band.hip: the forward and backward sweeps of the one-right-hand-side solve, the chunk
fetches of the many-right-hand-side solve, the staging loads of the trailing update) and
evaluates it for every thread of the first and last blocks, for every work-group count,
over shapes from one row to the subdomain sizes of the 3M-DOF flat laminate (about 90k
rows, half-bandwidth about 1900).  Every address must lie inside the matrix's storage
[0, n (B + 1)) plus BAND_PAD, every scratch index inside its segment.

(A load index one past these bounds faulted the GPU once, in the block-0 prefetch of the
many-right-hand-side solve; its indices are clamped since and this test pins them.)

The last test restates the factorisation launch's work-group numbering and waits and checks
that every wait is for a lower number.
"""

import numpy as np
import pytest

SB = 64            # solve block
SW = 8             # waves per solve work-group
RPW = 8            # forward rows per wave
UB = 32            # band rows in flight per wave (backward)
GMAX = 4           # work-groups per matrix, one right-hand side
DL = 8             # inverse-block entries per thread
MT = 512           # threads of the many-right-hand-side solve
AL = 8             # band-chunk entries per thread
NB = 64
BAND_PAD = 1024

SHAPES = [(1, 0), (2, 1), (63, 5), (64, 63), (65, 64), (127, 64), (128, 65), (129, 100),
          (300, 150), (1000, 63), (1000, 999), (4097, 700), (90783, 1899), (116493, 2433)]


def _blocks(nblk):
    """Blocks whose loads reach the extremes: the first and last few (the address
    expressions are monotone in the block index in between)."""
    return sorted(set(range(min(nblk, 6))) | set(range(max(0, nblk - 6), nblk)))


class Bounds:
    def __init__(self, n, B):
        self.n, self.B, self.ld = n, B, B + 1
        self.lo, self.hi = 0, n * (B + 1) + BAND_PAD     # factor storage incl. padding
        self.worst = 0

    def check(self, idx, what):
        idx = np.asarray(idx)
        if idx.size == 0:
            return
        assert idx.min() >= self.lo, (what, self.n, self.B, int(idx.min()))
        assert idx.max() < self.hi, (what, self.n, self.B, int(idx.max()), self.hi)
        self.worst = max(self.worst, int(idx.max()) - self.n * self.ld + 1)


def _single_rhs(n, B, G, bd):
    """k_band_solve_1 / band_solve_1_mat: forward and backward sweeps."""
    ld = B + 1
    nblk = (n + SB - 1) // SB
    w = np.arange(SW)[:, None, None]
    lane = np.arange(64)[None, :, None]
    r = np.arange(RPW)[None, None, :]
    for k in _blocks(nblk):
        i0 = k * SB
        kdone = max(k - G + 1, 0)
        done_end = kdone * SB
        ifirst = i0 + RPW * w
        rc = np.minimum(ifirst + r, n - 1)
        rowbase = rc * ld - rc + B                         # rp[r] = base + rc ld - rc + B
        # lane l loads V = 2 (FP64) or 4 (FP32) adjacent columns from c0 + V l (16 bytes),
        # 64 V columns per step, 512 columns per pass; the band (envelope) start, rounded
        # down to a 128-byte line of FP64 (16) or FP32 (32) entries: the first one is the
        # lower bound
        for V in (2, 4):
            US = 512 // (64 * V)
            start = np.maximum(ifirst - B, 0) // 32 * 32 + V * lane
            run = start < done_end + V * lane              # the c0 loop runs at all
            last = start + 512 * ((done_end + V * lane - 1 - start) // 512)
            shape = np.broadcast_shapes(rowbase.shape, run.shape)
            runf = np.broadcast_to(run, shape)
            for c0 in (start, last):
                assert (np.broadcast_to(c0 % V, run.shape)[run] == 0).all()   # aligned
                for u in range(US):
                    for e in range(V):
                        bd.check(np.broadcast_to(rowbase + c0 + 64 * V * u + e, shape)[runf],
                                 "forward band")
                        yi = np.broadcast_to(np.minimum(c0 + 64 * V * u + e, done_end - 1),
                                             run.shape)[run]
                        assert yi.size == 0 or (yi.min() >= 0 and yi.max() < nblk * SB)
        for o in range(GMAX - 1):                          # factor entries of blocks in flight
            cc = min(kdone + o, max(k - 1, 0)) * SB + lane
            bd.check(rowbase + cc, "forward in-flight")
            yi = min(kdone + o, max(k - 1, 0)) * SB + np.arange(64)
            assert yi.min() >= 0 and yi.max() < nblk * SB
        t = np.arange(512)
        d = k * SB * SB + t[:, None] + 512 * np.arange(DL)[None, :]
        assert d.min() >= 0 and d.max() < nblk * SB * SB
    rs = ld - 1
    for t in _blocks(nblk):
        kb = nblk - 1 - t
        i0 = kb * SB
        nb = min(SB, n - i0)
        rend = min(n, i0 + nb + B)
        kdone = kb + G
        done_beg = min(rend, kdone * SB)
        cidx = i0 + np.arange(64)[None, :]
        for wv in range(SW):
            r0s = list(range(done_beg + wv, rend, SW * UB))
            for r0 in (r0s[:1] + r0s[-1:]):
                # lane l loads the V columns from i0 + V (l mod 64 / V) of the rows
                # r0 + 8 (V v + l / (64 / V)), v < UB / V
                for V in (2, 4):
                    lpr = 64 // V
                    pr, hf = np.arange(64) % lpr, np.arange(64) // lpr
                    for v in range(UB // V):
                        rr = np.minimum(r0 + SW * (V * v + hf), rend - 1)
                        for e in range(V):
                            bd.check(rr * rs + B + i0 + V * pr + e, "backward band")
                zi = min(r0 + SW * (np.arange(64) % UB).max(), rend - 1)
                assert 0 <= zi < nblk * SB
            for o in range(GMAX - 1):
                for rr_ in range(RPW):
                    row = min((kb + 1 + o) * SB + wv + SW * rr_, n - 1)
                    bd.check(row * rs + B + cidx, "backward in-flight")
        zr = np.minimum((kb + 1 + np.arange(GMAX - 1))[:, None] * SB + np.arange(64)[None, :],
                        rend - 1)
        assert zr.min() >= 0 and zr.max() < nblk * SB


def _many_rhs(n, B, M, bd):
    """k_band_solve_m: the chunk fetches (band rows and solution rows) of both sweeps."""
    ld = B + 1
    rs = ld - 1
    nblk = (n + SB - 1) // SB
    wave = np.arange(MT) // 64
    lane = np.arange(MT) % 64
    YL = SB * M // MT

    def fetch(bwd, i0, kk):
        r0 = (kk * SB if bwd else i0) + wave
        c = (i0 if bwd else kk * SB) + lane
        for u in range(AL):
            bd.check(np.minimum(r0 + 8 * u, n - 1) * rs + B + c, "chunk band")
        yend = min(SB * M, (n - kk * SB) * M)
        assert yend > 0
        for u in range(YL):
            yi = kk * SB * M + np.minimum(np.arange(MT) + MT * u, yend - 1)
            assert yi.min() >= 0 and yi.max() < nblk * SB * M

    for k in _blocks(nblk):
        i0 = k * SB
        kfirst = max(i0 - B, 0) // SB
        count = k - kfirst
        if count > 0:
            for q in range(count + 2):                     # prefetches run two chunks ahead
                fetch(False, i0, kfirst + min(q, count - 1))
        nb = min(SB, n - i0)
        rows = np.minimum(i0 + np.arange(SB), n - 1)
        assert rows.max() < n
    for t in _blocks(nblk):
        kb = nblk - 1 - t
        i0 = kb * SB
        nb = min(SB, n - i0)
        klast = (min(n, i0 + nb + B) - 1) // SB
        count = klast - kb
        if count > 0:
            for q in range(count + 2):
                fetch(True, i0, klast - min(q, count - 1))


def _trailing_update(n, B, bd):
    """k_syrk_wide: the staging loads of both 128-row panel blocks for every tile of the
    update of a group's trailing window (tile columns two and on), in 32-bit offsets from
    the matrix start (its 16-byte loads read the same entries as one load per entry).  The
    panel launch k_chain loads only entries inside the band."""
    ld = B + 1
    rs = ld - 1
    rlast = n - 1
    T2, U2, GP = 128, 512, 4
    starts = list(range(0, n, GP * NB))
    for KW in (16, 32):                                     # FP64 and FP32 chunks
        kt = np.arange(U2) % KW
        i0 = np.arange(U2) // KW
        RP = U2 // KW
        PER = T2 // RP
        for k0 in starts[:3] + starts[-3:]:
            kj = min(GP * NB, n - k0)
            t0 = k0 + kj
            W = min(B, n - t0)
            if W <= 0:
                continue
            nt = (W + T2 - 1) // T2
            tiles = [(tr, ts) for ts in range(2, nt) for tr in range(ts, nt)]
            for tr, ts in tiles[:8] + tiles[-8:]:
                r0, s0 = t0 + tr * T2, t0 + ts * T2
                lo = r0 - B - k0
                kc_first = lo // KW * KW if lo > 0 else 0
                for kc in range(kc_first, kj, KW):
                    for u in range(PER):
                        r = np.minimum(r0 + i0 + RP * u, rlast)
                        ss = np.minimum(s0 + i0 + RP * u, rlast)
                        idx_r = r * rs + B + k0 + kt + kc
                        idx_s = ss * rs + B + k0 + kt + kc
                        assert idx_r.max() < 2 ** 31 and idx_s.max() < 2 ** 31
                        bd.check(idx_r, "trailing r")
                        bd.check(idx_s, "trailing s")


def _far_rows(n, B):
    """k_far: the 16-byte staging loads of the update of the rows below a group by the
    group's earlier panels.  Rows are not clamped: a row block that ends past the matrix
    reads up to 63 rows further, which the band allocation's padding (BAND_PAD + 128 rows)
    covers; offsets are 32-bit from the matrix start."""
    ld = B + 1
    rs = ld - 1
    CT, GP = 256, 4
    hi = n * ld + BAND_PAD + 128 * ld                       # the allocation's padding
    NR = (B + NB - 1) // NB + 1
    starts = list(range(0, n, GP * NB))
    for KC, VW in ((32, 2), (64, 4)):                       # FP64 and FP32 chunks
        tpr = KC // VW                                      # threads per staged row
        kt = np.arange(CT) % tpr * VW
        i0 = np.arange(CT) // tpr
        RP = CT // tpr
        PER = NB // RP
        for k0 in starts[:3] + starts[-3:]:
            for f in sorted(set(range(min(NR - 1, 3))) | set(range(max(0, NR - 4), NR - 1))):
                r0 = k0 + NB * (GP + f)
                if r0 >= n:
                    continue
                for p in range(1, GP):
                    c0 = k0 + NB * p
                    if c0 >= n or r0 > c0 + NB - 1 + B:
                        continue
                    lo = r0 - B                             # the envelope starts no earlier
                    kstart = k0 + (lo - k0) // KC * KC if lo > k0 else k0
                    kcs = list(range(kstart, c0, KC))
                    for kc in kcs[:1] + kcs[-1:]:
                        assert ((kc + kt) % VW == 0).all()  # 16-byte aligned (B % VW == 0)
                        for u in range(PER):
                            for row0 in (r0, c0):
                                idx = (row0 + i0 + RP * u) * rs + B + kc + kt
                                for e in range(VW):
                                    assert (idx + e).min() >= 0, ("far", n, B)
                                    assert (idx + e).max() < min(hi, 2 ** 31), ("far", n, B)


@pytest.mark.parametrize("n,B", SHAPES)
def test_band_kernel_loads_stay_in_the_padded_allocation(n, B):
    bd = Bounds(n, B)
    for G in range(1, GMAX + 1):
        _single_rhs(n, B, G, bd)
    for M in (8, 32):
        _many_rhs(n, B, M, bd)
    _trailing_update(n, B, bd)
    _far_rows(n, B)
    assert bd.worst <= 511                                  # far inside BAND_PAD


def test_padding_covers_the_worst_forward_overread():
    """The forward sweep of the one-right-hand-side solve reads furthest past the end: in
    the last block, rows clamped to n - 1 take columns up to done_end + 510."""
    bd = Bounds(1000, 63)
    _single_rhs(1000, 63, 1, bd)
    assert 400 < bd.worst <= 511


GP = 4             # panels per factorisation launch


def _chain_item(b, n_mat, NR):
    """The (panel p, matrix j, row block t) that k_chain's work-group number b works on."""
    if b < n_mat or NR == 1:
        return b // n_mat, b % n_mat, 0
    b -= n_mat
    for p in range(GP):
        m = NR - 1 + (p + 1 < GP)
        if b < n_mat * m:
            break
        b -= n_mat * m
    m = NR - 1 + (p + 1 < GP)
    j, o = divmod(b, m)
    if o == 0:
        return p, j, 1
    if p + 1 < GP and o == 1:
        return p + 1, j, 0
    return p, j, (o if p + 1 < GP else o + 1)


def _chain_waits(p, j, t, NR):
    """(panel, matrix, row block counted from the group start) of every flag the
    work-group waits for (restated from k_chain's steps 1 and 2b)."""
    tr = p + t
    w = []
    if p > 0:
        for q in range(p):
            if tr - q < NR:
                w.append((q, j, tr))
            if p - q < NR:
                w.append((q, j, p))
    if t > 0:
        w.append((p, j, p))
    return w


@pytest.mark.parametrize("n_mat,NR", [(1, 1), (1, 2), (3, 2), (2, 5), (16, 31), (64, 31),
                                      (64, 39)])
def test_factorisation_waits_are_for_earlier_numbers(n_mat, NR):
    """k_chain: the numbering covers every (panel, matrix, row block) once, every flag
    waited for is raised by exactly one work-group, and that work-group has a lower number.
    Work-groups take their numbers in the order they start, so the lowest-numbered
    unfinished one never waits: the launch always drains."""
    total = GP * n_mat * NR
    items = [_chain_item(b, n_mat, NR) for b in range(total)]
    assert sorted(items) == sorted((p, j, t) for p in range(GP) for j in range(n_mat)
                                   for t in range(NR))
    raised = {(p, j, p + t): b for b, (p, j, t) in enumerate(items)}
    assert len(raised) == total
    for b, (p, j, t) in enumerate(items):
        for f in _chain_waits(p, j, t, NR):
            assert f in raised, (b, f)
            assert raised[f] < b, (b, (p, j, t), f, raised[f])

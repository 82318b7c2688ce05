"""Model of the table-gradient partition used by the bin reduction (CPU).

The records of a step are grouped by gradient bin; ``k_bin_plan`` splits them over the G' reduction
blocks by cost (records plus a flush weight F for every non-empty bin), ``k_bin_reduce`` walks each
block's record range bin by bin (a bin wholly inside the range is flushed by that block, a bin cut
by a range boundary leaves its partial tile in slot 2j (the block's first bin) or 2j + 1 (its last)),
and ``k_bin_combine`` adds the slots of every cut bin in block order.  This file restates that
logic in Python, step for step with the kernels, and checks on thousands of random bin layouts that
every record is reduced exactly once, every non-empty bin is either flushed by one block or
combined once from exactly the slots that were written, and no slot is written twice.  It also
restates the wave scans that form the record offsets (``bin_row_scan``) and the plan's record and
cost starts (``k_bin_plan``) and checks them against plain prefix sums.  The GPU tests check the
kernels themselves (parity with the oracle, and bit-identical steps for different reduction grids).
"""
import numpy as np
import pytest


def _ceil_div(a, b):
    return -(-a // b)


def _plan(totals, G, F):
    """block_start[0..G'] and block_first_bin[0..G'-1] as k_bin_plan computes them."""
    n = len(totals)
    T = int(sum(totals))
    Ge = min(G, T)
    bs = np.zeros(n + 1, np.int64)
    bs[1:] = np.cumsum(totals)
    if T == 0:
        return T, 0, bs, np.zeros(1, np.int64), np.zeros(0, np.int64)
    cost = np.where(np.asarray(totals) > 0, np.asarray(totals, np.int64) + F, 0)
    CB = np.zeros(n + 1, np.int64)
    CB[1:] = np.cumsum(cost)
    C = int(CB[-1])
    block_start = np.full(Ge + 1, -1, np.int64)
    first_bin = np.full(Ge, -1, np.int64)
    for b in range(n):
        if totals[b] == 0:
            continue
        # blocks j whose cost boundary C j / G' falls in [CB[b], CB[b] + totals[b] + F)
        j0 = _ceil_div(int(CB[b]) * Ge, C)
        j1 = min(_ceil_div(int(CB[b + 1]) * Ge, C), Ge)
        for j in range(j0, j1):
            t = C * j // Ge - int(CB[b])
            if t < totals[b]:
                block_start[j] = bs[b] + t
                first_bin[j] = b
            else:   # inside the bin's flush share: the block starts at the next bin with records
                block_start[j] = bs[b] + totals[b]
                nb = b + 1
                while nb < n and totals[nb] == 0:
                    nb += 1
                first_bin[j] = min(nb, n - 1)
    block_start[Ge] = T
    return T, Ge, bs, block_start, first_bin


def _check(totals, G, F):
    n = len(totals)
    T, Ge, bs, st, bfb = _plan(totals, G, F)
    if T == 0:
        return 0, 0
    assert (st >= 0).all() and (np.diff(st) >= 0).all()
    cover = np.zeros(T, np.int32)
    writes, flushed = {}, {}
    # k_bin_reduce: each block walks its range segment by segment
    for jb in range(Ge):
        rs, re = st[jb], st[jb + 1]
        if rs >= re:
            continue                                       # an empty range
        first = bfb[jb]
        assert bs[first] <= rs < bs[first + 1], (jb, rs, first)
        pos, B = rs, first
        while pos < re:
            b_s, b_e = bs[B], bs[B + 1]
            if b_e <= pos:
                B += 1
                continue
            seg = min(re, b_e)
            cover[pos:seg] += 1
            if b_s < rs or b_e > re:                       # cut: partial tile to a slot
                writes.setdefault(B, []).append((jb, 2 * jb + (0 if B == first else 1)))
            else:
                flushed[B] = flushed.get(B, 0) + 1
            pos, B = seg, B + 1
    assert (cover == 1).all()
    slots = [s for v in writes.values() for _, s in v]
    assert len(slots) == len(set(slots))
    # k_bin_combine: block jb takes the bin holding record st[jb] when that bin starts in
    # [st[jb-1], st[jb]); it adds the slots of blocks jb-1 .. j1 (the last block reaching into the bin)
    combined = {}
    for jb in range(1, Ge):
        rs, rs_prev = st[jb], st[jb - 1]
        if rs >= T:
            continue
        B = bfb[jb]
        b_s, b_e = bs[B], bs[B + 1]
        if not (b_s < rs and b_s >= rs_prev):
            continue
        j1 = jb
        while j1 + 1 < Ge and st[j1 + 1] < b_e:
            j1 += 1
        used = [(jj, 2 * jj + (0 if bfb[jj] == B else 1)) for jj in range(jb - 1, j1 + 1) if st[jj] != st[jj + 1]]
        combined[B] = combined.get(B, 0) + 1
        assert sorted(used) == sorted(writes.get(B, [])), (B, used, writes.get(B))
    assert set(combined) == set(writes)
    assert all(v == 1 for v in combined.values())
    assert all(v == 1 for v in flushed.values())
    assert not (set(flushed) & set(writes))
    assert set(flushed) | set(writes) == {b for b in range(n) if totals[b] > 0}
    return len(writes), int((np.diff(st) == 0).sum())


def _layout(rng, kind, n):
    if kind == 0:
        return rng.integers(0, 50, n)
    if kind == 1:
        return rng.integers(0, 3, n)
    if kind == 2:
        return (rng.random(n) < 0.3) * rng.integers(1, 1000, n)
    if kind == 3:
        t = np.zeros(n, np.int64)
        t[rng.integers(0, n)] = rng.integers(1, 200)
        return t
    return rng.integers(0, 20000, n)


def test_partition_random_layouts():
    rng = np.random.default_rng(0)
    for trial in range(1500):
        n = int(rng.integers(1, 80))
        G = int(rng.integers(1, 48))
        F = int(rng.choice([0, 1, 3, 10, 100, 8192, 32768]))
        _check(list(map(int, _layout(rng, trial % 5, n))), G, F)


def test_partition_flush_weight_above_records():
    """F far above the record counts: many boundaries fall in flush shares, some ranges are empty."""
    rng = np.random.default_rng(1)
    empty = 0
    for _ in range(1000):
        n = int(rng.integers(1, 40))
        G = int(rng.integers(2, 64))
        F = int(rng.choice([100, 1000, 8192, 32768]))
        t = (rng.random(n) < 0.5) * rng.integers(1, 30, n)
        empty += _check(list(map(int, t)), G, F)[1]
    assert empty > 0   # the empty-range path was exercised


@pytest.mark.parametrize("F", [0, 32768])
def test_partition_ct256_like(F):
    """745 bins of 2^13 entries (heavy coarse bins first), 256 blocks."""
    rng = np.random.default_rng(2)
    t = np.concatenate([rng.integers(100000, 400000, 5), rng.integers(10000, 60000, 100),
                        rng.integers(30000, 70000, 640)])
    cut, _ = _check(list(map(int, t)), 256, F)
    assert 0 < cut < 256


def test_partition_empty_and_single():
    assert _check([0, 0, 0], 8, 32768) == (0, 0)
    _check([5], 1, 0)
    _check([5], 8, 32768)
    _check([0, 7, 0, 0, 3], 16, 1)


def _wave_scan_exclusive(vals, n_threads):
    """Exclusive prefix of per-thread values as the bin kernels form it: an inclusive scan inside
    each 64-lane wave (shifted partial sums, lanes below the shift keep theirs), the waves' totals
    through LDS, each thread adding the totals of the waves before its own."""
    vals = np.asarray(vals, np.int64)
    inc = vals.copy()
    lane = np.arange(n_threads) % 64
    o = 1
    while o < 64:
        shifted = np.zeros_like(inc)
        shifted[o:] = inc[:-o]
        inc = inc + np.where(lane >= o, shifted, 0)
        o <<= 1
    wave_tot = inc[63::64]
    before = np.concatenate([[0], np.cumsum(wave_tot)[:-1]])[np.arange(n_threads) // 64]
    return before + inc - vals, int(wave_tot.sum())


@pytest.mark.parametrize("grid", [1, 7, 255, 256, 512, 1000, 2048])
def test_row_scan_offsets(grid):
    """bin_row_scan: 256 threads, each summing `per` consecutive blocks' counts, then the wave scan;
    the offsets of every (bin, block) must be the plain exclusive prefix of the counts."""
    rng = np.random.default_rng(grid)
    counts = rng.integers(0, 600, grid)
    counts[rng.random(grid) < 0.2] = 0
    per = _ceil_div(grid, 256)
    s = np.array([counts[t * per:min(grid, t * per + per)].sum() for t in range(256)])
    ex, total = _wave_scan_exclusive(s, 256)
    rel = np.zeros(grid, np.int64)
    for t in range(256):
        run = ex[t]
        for w in range(t * per, min(grid, t * per + per)):
            rel[w] = run
            run += counts[w]
    assert total == counts.sum()
    assert np.array_equal(rel, np.concatenate([[0], np.cumsum(counts)[:-1]]))


@pytest.mark.parametrize("n_bins", [1, 29, 745, 1024, 3000])
def test_plan_scan_starts(n_bins):
    """k_bin_plan: 1024 threads, each summing its bins' records and costs (records + F per
    non-empty bin), then the wave scans; every thread's record and cost start must be the exclusive
    prefix over the bins before its own, and the totals the sums."""
    rng = np.random.default_rng(n_bins)
    F = 32768
    tot = rng.integers(0, 60000, n_bins)
    tot[rng.random(n_bins) < 0.1] = 0
    per = _ceil_div(n_bins, 1024)
    rec = np.array([tot[t * per:min(n_bins, t * per + per)].sum() for t in range(1024)])
    cost = np.array([(tot[t * per:min(n_bins, t * per + per)] + F * (tot[t * per:min(n_bins, t * per + per)] > 0)).sum()
                     for t in range(1024)])
    rex, T = _wave_scan_exclusive(rec, 1024)
    cex, C = _wave_scan_exclusive(cost, 1024)
    assert T == tot.sum() and C == (tot + F * (tot > 0)).sum()
    assert np.array_equal(rex, np.concatenate([[0], np.cumsum(rec)[:-1]]))
    assert np.array_equal(cex, np.concatenate([[0], np.cumsum(cost)[:-1]]))

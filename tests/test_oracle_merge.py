"""Pins of the oracle's superparticle merge/split: the paper's worked example (1000
particles uniform in a cell with weights uniform on 1..100 merged to 64 particles whose
weights differ by at most one), splitting a single superparticle, conservation of
weight and weighted centroid, leaf counts, and the weight median of eq. weight_median
against brute force on tiny sets."""
import itertools

import numpy as np
import pytest


def test_paper_example_1000_to_64(orc):
    rng = np.random.default_rng(2023)
    m = 1000
    off = rng.random((m, 3))
    w = rng.integers(1, 101, size=m).astype(np.uint64)
    ids = np.arange(m, dtype=np.uint64)
    lo, lw, li = orc.merge_cell(64, off, w, ids, cell=5, step=9)
    assert len(lw) == 64
    assert int(lw.max()) - int(lw.min()) <= 1
    assert int(lw.sum()) == int(w.sum())
    cen = (off * w[:, None].astype(float)).sum(0)
    assert np.allclose((lo * lw[:, None].astype(float)).sum(0), cen, rtol=1e-12)
    assert np.all(lo >= 0) and np.all(lo < 1)
    assert len(set(li.tolist())) == 64 and all(int(x) >> 62 == 3 for x in li)


def test_split_single_superparticle(orc):
    off = np.array([[0.2, 0.7, 0.4]])
    lo, lw, li = orc.merge_cell(32, off, np.array([1000], dtype=np.uint64),
                                np.array([77], dtype=np.uint64))
    assert len(lw) == 32
    assert sorted(set(lw.tolist())) == [31, 32]
    assert int((lw == 32).sum()) == 8 and int((lw == 31).sum()) == 24
    assert np.allclose(lo, off)


@pytest.mark.parametrize("m,wmax,nppc", [(10, 1, 32), (5, 3, 32), (40, 1, 32), (200, 50, 32),
                                         (33, 1, 32), (7, 1000, 16), (100, 1, 8)])
def test_invariants(orc, m, wmax, nppc):
    rng = np.random.default_rng(m * 1000 + wmax)
    off = rng.random((m, 3))
    w = rng.integers(1, wmax + 1, size=m).astype(np.uint64)
    ids = rng.permutation(m).astype(np.uint64) * np.uint64(3)
    lo, lw, li = orc.merge_cell(nppc, off, w, ids)
    W = int(w.sum())
    assert len(lw) == min(nppc, W)
    assert int(lw.sum()) == W
    assert np.all(lw >= 1)
    cen = (off * w[:, None].astype(float)).sum(0)
    assert np.allclose((lo * lw[:, None].astype(float)).sum(0), cen, rtol=1e-12)
    if nppc & (nppc - 1) == 0 and W >= nppc:
        assert int(lw.max()) - int(lw.min()) <= 1


def _median_brute(ws):
    """Smallest 1-based p' with sum_{p<p'} w + w_p' > sum_{p>p'} w, by enumeration."""
    M = len(ws)
    for pp in range(1, M + 1):
        if sum(ws[:pp - 1]) + ws[pp - 1] > sum(ws[pp:]):
            return pp
    raise AssertionError


def test_first_split_matches_bruteforce(orc):
    """Two leaves: the split of the root must put floor(W/2) / ceil(W/2) on the two
    sides exactly as the brute-force median with the physical/superparticle rule."""
    rng = np.random.default_rng(11)
    for trial in range(300):
        m = int(rng.integers(1, 7))
        ws = rng.integers(1, 6, size=m).tolist()
        if sum(ws) < 2:
            continue
        # offsets spread along x only, so the split axis is x and the order is by x
        xs = rng.permutation(m) / m + 0.01
        off = np.stack([xs, np.full(m, 0.5), np.full(m, 0.5)], 1)
        order = np.argsort(xs)
        wsorted = [ws[i] for i in order]
        pp = _median_brute(wsorted)
        Wl, wm, Wr = sum(wsorted[:pp - 1]), wsorted[pp - 1], sum(wsorted[pp:])
        if wm == 1:
            left = Wl + 1 if Wl <= Wr else Wl
        else:
            left = (Wl + wm + Wr) // 2
        lo, lw, li = orc.merge_cell(2, off, np.array(ws, dtype=np.uint64),
                                    np.arange(m, dtype=np.uint64))
        assert len(lw) == 2
        assert int(lw[0]) == left
        assert int(lw[0] + lw[1]) == sum(ws)
        assert abs(int(lw[0]) - int(lw[1])) <= 1


def test_largest_extent_axis(orc):
    # particles spread along y, two groups: the first split must separate by y
    off = np.array([[0.5, 0.1, 0.5], [0.52, 0.12, 0.5], [0.5, 0.9, 0.5], [0.48, 0.88, 0.51]])
    lo, lw, li = orc.merge_cell(2, off, np.ones(4, dtype=np.uint64), np.arange(4, dtype=np.uint64))
    assert sorted(np.round(lo[:, 1], 2).tolist()) == [0.11, 0.89]

"""The counting sort by cell as a kernel-level entry point, through the C ABI, against
its plain definition: the live particles (w > 0, cell < ncell) grouped by ascending
cell, start = the exclusive prefix of the per-cell counts, each cell's particles exactly
those of the input (compared as sets, the order inside a cell being unspecified)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def itk():
    import torch
    assert torch.cuda.is_available()
    from paper_2307_01797_amd import itokmc
    itokmc.lib()
    return itokmc


def make_input(rng, n, ncell, dead_frac=0.1, bad_frac=0.01, sorted_frac=0.5):
    cell = rng.integers(0, ncell, size=n).astype(np.uint32)
    k = int(n * sorted_frac)        # part of the input already grouped (long runs)
    cell[:k] = np.sort(cell[:k])
    bad = rng.random(n) < bad_frac
    cell[bad] = ncell + rng.integers(0, 1000, size=bad.sum()).astype(np.uint32)
    w = rng.integers(1, 1 << 20, size=n).astype(np.uint32)
    w[rng.random(n) < dead_frac] = 0
    off = rng.random((n, 3)) * 0.999
    ids = rng.permutation(n).astype(np.uint64) * np.uint64(7919) + np.uint64(3)
    return cell, off, w, ids


def check_sorted(out, cell, off, w, ids, ncell, prec):
    start, c2, o2, w2, i2 = out
    live = (w > 0) & (cell < ncell)
    cnt = np.bincount(cell[live].astype(np.int64), minlength=ncell)
    want_start = np.concatenate([[0], np.cumsum(cnt)]).astype(np.uint64)
    assert np.array_equal(start.astype(np.uint64), want_start)
    assert len(i2) == live.sum()
    assert np.all(np.diff(c2.astype(np.int64)) >= 0)
    # within each cell the same particles: compare sorted by (cell, id)
    a = np.lexsort((ids[live], cell[live]))
    b = np.lexsort((i2, c2))
    assert np.array_equal(c2[b], cell[live][a])
    assert np.array_equal(i2[b], ids[live][a])
    assert np.array_equal(w2[b], w[live][a])
    ref = off[live][a]
    if prec == "fp32":
        ref = ref.astype(np.float32).astype(np.float64)
    assert np.array_equal(o2[b], ref)


@pytest.mark.parametrize("n,ncell,prec", [(100_000, 32 ** 3, "fp32"), (250_001, 48 * 40 * 37, "fp64"),
                                          (3_000_000, 1 << 20, "fp32"), (0, 1000, "fp32"),
                                          (5000, 1 << 24, "fp32"), (1, 1, "fp64")])
def test_sort_by_cell_matches_definition(itk, n, ncell, prec):
    rng = np.random.default_rng(n + ncell)
    cell, off, w, ids = make_input(rng, n, ncell)
    print(f"sort n={n} ncell={ncell} {prec}", flush=True)
    out = itk.sort_by_cell(cell, off, w, ids, ncell, precision=prec)
    check_sorted(out, cell, off, w, ids, ncell, prec)


def test_sort_rejects_bad_arguments(itk):
    import ctypes
    L = itk.lib()
    assert L.itokmc_sort_workspace_bytes(10, 0) == 0
    assert L.itokmc_sort_workspace_bytes(10, (1 << 24) + 1) == 0
    z = [None] * 14
    assert L.itokmc_sort_by_cell(0, 10, 100, *z, None, 0, None) == itk.EINVAL
    assert L.itokmc_sort_by_cell(5, 0, 100, *z, None, 0, None) == itk.EINVAL

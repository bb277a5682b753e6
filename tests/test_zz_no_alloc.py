"""The no-allocation sort (its scratch a file-scope device array) against the sort
that takes a caller workspace: the same start array and the same particles in each
cell, on two calls in a row, the second with a smaller input (the array keeps the first
call's contents, so the counters must be cleared on every call); sizes beyond the
array's 32 MiB are rejected with ECAPACITY."""
import numpy as np
import pytest

from test_gpu_sort import check_sorted, make_input

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def itk():
    import torch
    assert torch.cuda.is_available()
    from paper_2307_01797_amd import itokmc
    itokmc.lib()
    return itokmc


def test_noalloc_matches_workspace_sort_twice(itk):
    rng = np.random.default_rng(77)
    for n, ncell, prec in ((2_000_000, 1 << 20, "fp32"), (30_000, 20 * 17 * 13, "fp64")):
        print(f"noalloc n={n} ncell={ncell} {prec}", flush=True)
        cell, off, w, ids = make_input(rng, n, ncell)
        a = itk.sort_by_cell(cell, off, w, ids, ncell, precision=prec, noalloc=True)
        b = itk.sort_by_cell(cell, off, w, ids, ncell, precision=prec, noalloc=False)
        assert np.array_equal(a[0], b[0])
        for out in (a, b):
            check_sorted(out, cell, off, w, ids, ncell, prec)


def test_noalloc_rejects_sizes_beyond_scratch(itk):
    import ctypes
    L = itk.lib()
    n, ncell = 8_000_000, 1 << 22
    assert L.itokmc_sort_workspace_bytes(n, ncell) > 32 << 20
    p = [ctypes.c_void_p(16)] * 14   # never dereferenced: the size check comes first
    assert L.itokmc_sort_by_cell_noalloc(0, n, ncell, *p, None) == itk.ECAPACITY

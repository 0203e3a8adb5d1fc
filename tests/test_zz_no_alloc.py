"""spc_matrix_features_noalloc (the entry point that allocates nothing)
against spc_matrix_features, through the C ABI: identical features and block
counts on two calls in a row, the second on a smaller matrix (the fixed
scratch keeps the first call's contents), and a size beyond the scratch's
limit refused before any device work."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_1801_01134_amd import _binding as Bd
from paper_1801_01134_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _features(fn, A):
    rp = torch.from_numpy(A.rowptr).cuda()
    ci = torch.from_numpy(A.colidx if A.nnz else np.zeros(1, np.int32)).cuda()
    f = (ctypes.c_float * 16)()
    nb = (ctypes.c_int64 * 6)()
    Bd.check(fn(A.n_rows, A.n_cols, A.nnz, Bd._ptr(rp), Bd._ptr(ci), f, nb, Bd.stream_ptr()))
    return np.array(list(f), dtype=np.float32), np.array(list(nb), dtype=np.int64)


def test_noalloc_features_equal_allocating_entry_point():
    L = Bd.lib()
    big = synth.stencil27(40)                         # 64,000 rows: 32 partial blocks
    small = synth.powerlaw(3001, 3001, seed=2)        # 3,001 rows: 2 partial blocks
    for name, A in (("stencil40", big), ("powerlaw3001", small)):
        say(f"[noalloc] {name} n={A.n_rows} nnz={A.nnz}")
        f0, n0 = _features(L.spc_matrix_features, A)
        f1, n1 = _features(L.spc_matrix_features_noalloc, A)
        assert np.array_equal(f0.view(np.uint32), f1.view(np.uint32)), (name, f0, f1)
        assert np.array_equal(n0, n1), name


def test_noalloc_refuses_sizes_beyond_its_scratch():
    L = Bd.lib()
    cap = int(L.spc_matrix_features_noalloc_max_rows())
    assert cap >= 16_000_000
    f = (ctypes.c_float * 16)()
    # pointers are never dereferenced: the size check comes first
    st = L.spc_matrix_features_noalloc(cap + 1, 10, 0, ctypes.c_void_p(4096), None, f, None, None)
    assert st == -8                                   # SPC_ERR_CAPACITY
    assert b"at most" in L.spc_last_error()

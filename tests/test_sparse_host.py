"""Host-side index build of the sparse form (cp_sparse_index): no GPU needed,
the call touches no device."""
import ctypes
import os

import numpy as np
import pytest

from paper_1111_6091_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1111_6091_amd", "libcpamg.so")
needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libcpamg.so not built")


def _index(idx, dims):
    from paper_1111_6091_amd import _lib
    lib = _lib.load()
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
    nnz, N = idx.shape if idx.ndim == 2 else (0, len(dims))
    dd = (ctypes.c_int64 * len(dims))(*dims)
    rowptr = np.full(sum(d + 1 for d in dims), -7, dtype=np.int64)
    perm = np.full(max(1, N * nnz), -7, dtype=np.int32)
    rc = lib.cp_sparse_index(None, len(dims), dd, nnz, idx.ctypes.data_as(ctypes.c_void_p),
                             rowptr.ctypes.data_as(ctypes.c_void_p), perm.ctypes.data_as(ctypes.c_void_p))
    return rc, rowptr, perm


@needs_lib
@pytest.mark.parametrize("case", ["laplacian", "random"])
def test_orderings_group_entries_by_index(case):
    if case == "laplacian":
        idx, _, dims = synth.laplacian_coo(2, 5)
    else:
        rng = np.random.default_rng(3)
        dims = (7, 1, 9, 4)
        P = int(np.prod(dims))
        lin = rng.choice(P, size=60, replace=False)   # unsorted on purpose
        idx = np.stack(np.unravel_index(lin, dims, order="F"), axis=1).astype(np.int32)
    rc, rowptr, perm = _index(idx, dims)
    assert rc == 0
    nnz = idx.shape[0]
    off = 0
    for m, d in enumerate(dims):
        rp = rowptr[off:off + d + 1]
        pm = perm[m * nnz:(m + 1) * nnz]
        off += d + 1
        assert rp[0] == 0 and rp[-1] == nnz
        assert np.array_equal(np.diff(rp), np.bincount(idx[:, m], minlength=d))
        assert np.array_equal(np.sort(pm), np.arange(nnz))
        for i in range(d):
            ids = pm[rp[i]:rp[i + 1]]
            assert np.all(idx[ids, m] == i)
            assert np.all(np.diff(ids) > 0)   # increasing entry id within an index


@needs_lib
def test_bad_input_is_rejected():
    from paper_1111_6091_amd._lib import CP_ERR_INVALID, CP_ERR_SHAPE
    dims = (3, 4)
    assert _index([[0, 0], [2, 4]], dims)[0] == CP_ERR_INVALID        # index outside its extent
    assert _index([[0, 0], [-1, 1]], dims)[0] == CP_ERR_INVALID       # negative index
    assert _index([[1, 2], [0, 0], [1, 2]], dims)[0] == CP_ERR_INVALID  # same tuple twice
    assert _index(np.zeros((0, 2)), dims)[0] == CP_ERR_SHAPE          # no entries
    assert _index([[0] * 9], (2,) * 9)[0] == CP_ERR_SHAPE             # order above the maximum

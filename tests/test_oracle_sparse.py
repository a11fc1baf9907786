"""The sparse test problem of Section 6.2 and the oracle's MTTKRP over stored
nonzeros: the Laplacian tensor against the paper's Kronecker-sum matrix, the
coarsening thresholds against Table 3's level counts, and the coordinate-form
MTTKRP against the dense definition and brute force."""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import amg, cp
from paper_1111_6091_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _kron_sum_matrix(d, s):
    """sum_k I_{s^(d-k)} (x) D (x) I_{s^(k-1)} with D = tridiag(-1, 2, -1)."""
    D = 2.0 * np.eye(s) - np.eye(s, k=1) - np.eye(s, k=-1)
    Zm = np.zeros((s ** d, s ** d))
    for k in range(1, d + 1):
        Zm += np.kron(np.eye(s ** (d - k)), np.kron(D, np.eye(s ** (k - 1))))
    return Zm


@pytest.mark.parametrize("d,s", [(2, 4), (2, 5), (3, 3), (4, 2)])
def test_laplacian_matches_kronecker_sum(d, s):
    """Column-major reshape of the s^d x s^d Kronecker-sum matrix."""
    idx, vals, shape = synth.laplacian_coo(d, s)
    Zd = synth.coo_to_dense(idx, vals, shape)
    ref = _kron_sum_matrix(d, s).reshape(shape, order="F")
    assert np.array_equal(Zd, ref)
    assert idx.shape[0] == np.count_nonzero(ref) == s ** d + 2 * d * (s - 1) * s ** (d - 1)
    # stored in increasing linear order (mode 1 fastest), no index twice
    lin = np.ravel_multi_index(tuple(idx.T.astype(np.int64)), shape, order="F")
    assert np.all(np.diff(lin) > 0)


def test_laplacian_symmetries():
    """The matrix is symmetric (swap the row and column digit modes) and the
    grid directions are interchangeable (permute the digit pairs together)."""
    d, s = 3, 4
    Z = synth.coo_to_dense(*synth.laplacian_coo(d, s))
    assert np.array_equal(Z, np.transpose(Z, (3, 4, 5, 0, 1, 2)))
    assert np.array_equal(Z, np.transpose(Z, (1, 0, 2, 4, 3, 5)))
    assert np.array_equal(Z, np.transpose(Z, (2, 1, 0, 5, 4, 3)))
    # the row of an interior grid point: 2d on the diagonal, 2d neighbours of -1
    i = (1, 2, 1)
    row = Z[i]
    assert row[i] == 2.0 * d and np.sum(row == -1.0) == 2 * d and np.count_nonzero(row) == 2 * d + 1


def test_coarsening_threshold_reproduces_table3_levels():
    with open(os.path.join(HERE, "golden", "table3_laplacian_levels.json")) as f:
        rows = json.load(f)["tests"]
    assert len(rows) == 11
    for row in rows:
        N, s, R = row["N"], row["s"], row["R"]
        assert synth.LAPLACIAN_TESTS[row["test"]] == (N, s, R)
        coarsest = [synth.LAPLACIAN_COARSEST[N]] * N
        assert min(coarsest) >= R   # Section 4.5: I_{n,coarsest} >= R
        assert amg.n_levels((s,) * N, coarsest) == row["levs"], row


@pytest.mark.parametrize("shape,nnz", [((3, 4, 2), 9), ((2, 3, 2, 4), 20), ((5, 2, 3), 30)])
def test_mttkrp_coo_brute_force(shape, nnz):
    """Elementwise sum over the stored entries, and the dense definition on the
    densified tensor, for random sparsity patterns."""
    rng = np.random.default_rng(sum(shape) + nnz)
    P = int(np.prod(shape))
    lin = np.sort(rng.choice(P, size=nnz, replace=False))
    idx = np.stack(np.unravel_index(lin, shape, order="F"), axis=1).astype(np.int32)
    vals = rng.standard_normal(nnz)
    R = 3
    A = [rng.standard_normal((I, R)) for I in shape]
    Zd = synth.coo_to_dense(idx, vals, shape)
    for n in range(len(shape)):
        M = cp.mttkrp_coo(idx, vals, shape, A, n)
        B = np.zeros_like(M)
        for k in range(nnz):
            for r in range(R):
                t = vals[k]
                for m in range(len(shape)):
                    if m != n:
                        t *= A[m][idx[k, m], r]
                B[idx[k, n], r] += t
        assert np.allclose(M, B, rtol=1e-14, atol=1e-14)
        assert np.allclose(M, cp.mttkrp(Zd, A, n), rtol=1e-13, atol=1e-13)


def test_mttkrp_coo_laplacian_closed_form():
    """Factors of ones (R = 1): M^(n)(i) is the sum of the mode-n slice i.  For
    a digit mode k of the Laplacian the term of direction k gives the row sum
    of D at i (1 at the two ends, 0 inside) times s^(d-1), and each of the other
    d - 1 directions gives the sum of all entries of D (2) times s^(d-2)."""
    for d, s in [(2, 6), (3, 5)]:
        idx, vals, shape = synth.laplacian_coo(d, s)
        Zd = synth.coo_to_dense(idx, vals, shape)
        A = [np.ones((s, 1)) for _ in shape]
        expect = np.full(s, 2.0 * (d - 1) * s ** (d - 2))
        expect[0] += s ** (d - 1)
        expect[-1] += s ** (d - 1)
        for n in range(2 * d):
            M = cp.mttkrp_coo(idx, vals, shape, A, n)
            assert np.array_equal(M[:, 0], expect), (d, s, n)
            sums = np.sum(np.moveaxis(Zd, n, 0).reshape(s, -1), axis=1)
            assert np.array_equal(M[:, 0], sums)


def test_multilevel_on_laplacian_converges_to_als_minimum():
    """'Multilevel' and 'Multilevel + FMG' (Section 6.1) on the N = 4, s = 10
    Laplacian, R = 2, two levels (10 -> 5): both reach g < 1e-10 at the fit that
    standalone ALS from the same boot factors converges to."""
    c = synth.laplacian_case(4, 10, 2)
    Z = synth.coo_to_dense(c["idx"], c["vals"], c["shape"])
    crs = [5] * 4
    A, info = amg.multilevel(Z, c["boot"], c["tfms"], crs, setup=amg.SETUP_PARAMS_NO_NT,
                             fas=amg.FAS_PARAMS)
    assert info["levels"] == 2 and info["solve"][-1] < 1e-10
    B, h = cp.als(Z, c["boot"], max_sweeps=5000, fit_tol=None, g_tol=1e-10)
    assert h["g"][-1] < 1e-10
    assert abs(cp.fit(Z, A) - cp.fit(Z, B)) < 1e-10
    cs = [np.random.default_rng(c["seed"] + 1).random((5, 2)) for _ in range(4)]
    A2, info2 = amg.multilevel_fmg(Z, c["boot"], c["tfms"], crs, cs, setup=amg.SETUP_PARAMS_NO_NT,
                                   fas=amg.FAS_PARAMS)
    assert info2["solve"][-1] < 1e-10
    assert abs(cp.fit(Z, A2) - cp.fit(Z, B)) < 1e-10

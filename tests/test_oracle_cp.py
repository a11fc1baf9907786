"""Pins of the CP/ALS oracle against brute force, closed forms and invariants.

Each check is computed by a route that does not reuse the oracle function it
tests (explicit index loops, Kronecker products from numpy, finite differences,
least-squares solvers), so that a dropped term, a wrong index order or a
transposed operand in the oracle fails one of them.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import cp
from paper_1111_6091_amd import synth


def rand_factors(rng, dims, R):
    return [rng.standard_normal((d, R)) for d in dims]


def brute_full(A):
    dims = [a.shape[0] for a in A]
    R = A[0].shape[1]
    T = np.zeros(dims)
    for idx in itertools.product(*[range(d) for d in dims]):
        s = 0.0
        for r in range(R):
            p = 1.0
            for n, i in enumerate(idx):
                p *= A[n][i, r]
            s += p
        T[idx] = s
    return T


def brute_mttkrp(Z, A, n):
    dims = Z.shape
    R = A[0].shape[1]
    M = np.zeros((dims[n], R))
    for idx in itertools.product(*[range(d) for d in dims]):
        for r in range(R):
            p = Z[idx]
            for m, i in enumerate(idx):
                if m != n:
                    p *= A[m][i, r]
            M[idx[n], r] += p
    return M


def brute_objective(Z, A):
    D = Z - brute_full(A)
    return 0.5 * float(np.sum(D ** 2))


def brute_mode_product(Z, M, n):
    dims = list(Z.shape)
    out_dims = dims.copy()
    out_dims[n] = M.shape[0]
    X = np.zeros(out_dims)
    for idx in itertools.product(*[range(d) for d in out_dims]):
        s = 0.0
        for i in range(dims[n]):
            src = list(idx)
            src[n] = i
            s += M[idx[n], i] * Z[tuple(src)]
        X[idx] = s
    return X


@pytest.mark.parametrize("dims", [(3, 4, 2), (2, 3, 4, 5)])
def test_unfold_column_order_brute(dims):
    rng = np.random.default_rng(0)
    Z = rng.standard_normal(dims)
    N = len(dims)
    for n in range(N):
        Zn = cp.unfold(Z, n)
        for idx in itertools.product(*[range(d) for d in dims]):
            col, J = 0, 1
            for k in range(N):
                if k == n:
                    continue
                col += idx[k] * J
                J *= dims[k]
            assert Zn[idx[n], col] == Z[idx]
        np.testing.assert_array_equal(cp.fold(Zn, n, dims), Z)


@pytest.mark.parametrize("dims", [(3, 4, 2), (2, 3, 2, 3)])
def test_matricized_product_identity(dims):
    """eq. (5): X = Z x_1 A1 ... x_N AN  <=>  X_(n) = A^(n) Z_(n) (A^(N) kron ... kron A^(1))^T."""
    rng = np.random.default_rng(1)
    Z = rng.standard_normal(dims)
    Ms = [rng.standard_normal((d + 1, d)) for d in dims]
    X = Z
    for n, M in enumerate(Ms):
        X = brute_mode_product(X, M, n)
    N = len(dims)
    for n in range(N):
        K = np.ones((1, 1))
        for m in reversed(range(N)):
            if m != n:
                K = np.kron(K, Ms[m])
        np.testing.assert_allclose(cp.unfold(X, n), Ms[n] @ cp.unfold(Z, n) @ K.T,
                                   rtol=1e-12, atol=1e-12)
    # the oracle's mode product agrees with the brute-force one, and products commute
    Y1 = cp.mode_product(cp.mode_product(Z, Ms[0], 0), Ms[1], 1)
    Y2 = cp.mode_product(cp.mode_product(Z, Ms[1], 1), Ms[0], 0)
    np.testing.assert_allclose(Y1, Y2, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(Y1, brute_mode_product(brute_mode_product(Z, Ms[0], 0), Ms[1], 1),
                               rtol=1e-13, atol=1e-13)


def test_khatri_rao_definition_and_kkr_identity():
    """Columns are Kronecker products; eq. (4): A1B1 (.) A2B2 (.) A3B3 = (A1 kron A2 kron A3)(B1 (.) B2 (.) B3)."""
    rng = np.random.default_rng(2)
    R = 3
    Bs = [rng.standard_normal((d, R)) for d in (2, 3, 4)]
    As = [rng.standard_normal((d + 2, d)) for d in (2, 3, 4)]
    KR = cp.khatri_rao(Bs)
    for r in range(R):
        np.testing.assert_array_equal(KR[:, r], np.kron(np.kron(Bs[0][:, r], Bs[1][:, r]), Bs[2][:, r]))
    lhs = cp.khatri_rao([a @ b for a, b in zip(As, Bs)])
    rhs = np.kron(np.kron(As[0], As[1]), As[2]) @ KR
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dims,R", [((3, 4, 5), 2), ((2, 3, 4, 5), 3), ((5, 2, 3), 4)])
def test_mttkrp_brute_force(dims, R):
    rng = np.random.default_rng(3)
    Z = rng.standard_normal(dims)
    A = rand_factors(rng, dims, R)
    for n in range(len(dims)):
        np.testing.assert_allclose(cp.mttkrp(Z, A, n), brute_mttkrp(Z, A, n), rtol=1e-13, atol=1e-13)


def test_mttkrp_rank_one_closed_form():
    rng = np.random.default_rng(4)
    a, b, c = rng.standard_normal(5), rng.standard_normal(4), rng.standard_normal(3)
    Z = np.multiply.outer(np.multiply.outer(a, b), c)
    A = rand_factors(rng, (5, 4, 3), 3)
    expect = np.outer(a, (b @ A[1]) * (c @ A[2]))
    np.testing.assert_allclose(cp.mttkrp(Z, A, 0), expect, rtol=1e-13, atol=1e-13)
    expect3 = np.outer(c, (a @ A[0]) * (b @ A[1]))
    np.testing.assert_allclose(cp.mttkrp(Z, A, 2), expect3, rtol=1e-13, atol=1e-13)


def test_full_and_objectives():
    rng = np.random.default_rng(5)
    dims, R = (3, 4, 5), 3
    A = rand_factors(rng, dims, R)
    Z = rng.standard_normal(dims)
    np.testing.assert_allclose(cp.full(A), brute_full(A), rtol=1e-13, atol=1e-13)
    f = cp.objective(Z, A)
    assert f == pytest.approx(brute_objective(Z, A), rel=1e-13)
    M = brute_mttkrp(Z, A, 2)
    G = [a.T @ a for a in A]
    ff = cp.objective_fused(float(np.sum(Z ** 2)), A[2], M, G)
    assert ff == pytest.approx(f, rel=1e-11)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(6)
    dims, R = (3, 4, 2), 2
    A = rand_factors(rng, dims, R)
    Z = rng.standard_normal(dims)
    G = cp.gradient(Z, A)
    h = 1e-6
    for n in range(3):
        for i in range(dims[n]):
            for r in range(R):
                Ap = [a.copy() for a in A]
                Am = [a.copy() for a in A]
                Ap[n][i, r] += h
                Am[n][i, r] -= h
                fd = (brute_objective(Z, Ap) - brute_objective(Z, Am)) / (2 * h)
                assert G[n][i, r] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    g = cp.grad_norm(Z, A)
    assert g == pytest.approx(math.sqrt(sum(float(np.sum(x * x)) for x in G)) / np.linalg.norm(Z), rel=1e-14)


def test_gamma_is_hadamard_of_other_grams():
    rng = np.random.default_rng(7)
    A = rand_factors(rng, (4, 5, 6, 3), 3)
    Gs = cp.grams(A)
    for n in range(4):
        expect = np.ones((3, 3))
        for m in range(4):
            if m != n:
                for r in range(3):
                    for s in range(3):
                        expect[r, s] *= sum(A[m][i, r] * A[m][i, s] for i in range(A[m].shape[0]))
        np.testing.assert_allclose(cp.gamma(Gs, n), expect, rtol=1e-13)
        # symmetric positive definite when the factors have full rank
        assert np.all(np.linalg.eigvalsh(cp.gamma(Gs, n)) > 0)


def test_solve_gamma_spd_and_singular():
    rng = np.random.default_rng(8)
    R = 4
    X = rng.standard_normal((6, R))
    S = rng.standard_normal((R, R))
    Gam = S @ S.T + R * np.eye(R)
    B = rng.standard_normal((6, R))
    Xs, fb = cp.solve_gamma(B, Gam, return_info=True)
    assert not fb
    np.testing.assert_allclose(Xs, np.linalg.solve(Gam.T, B.T).T, rtol=1e-12)
    # singular Gamma (a factor with a zero column makes a zero row/column)
    A = rand_factors(rng, (5, 6, 7), R)
    A[1][:, 2] = 0.0
    Gs = cp.grams(A)
    Gs0 = cp.gamma(Gs, 0)
    Xp, fb = cp.solve_gamma(B, Gs0, return_info=True)
    assert fb
    np.testing.assert_allclose(Xp, B @ np.linalg.pinv(Gs0, rcond=R * np.finfo(float).eps),
                               rtol=1e-10, atol=1e-12)
    del X


def test_gauss_seidel_properties():
    rng = np.random.default_rng(9)
    R = 5
    S = rng.standard_normal((R, R))
    Gam = S @ S.T + 0.5 * np.eye(R)
    B = rng.standard_normal((7, R))
    X0 = rng.standard_normal((7, R))
    exact = np.linalg.solve(Gam, B.T).T
    # GS(inf) converges to the Cholesky solution for SPD Gamma
    np.testing.assert_allclose(cp.gauss_seidel(X0, Gam, B, 4000), exact, rtol=1e-9, atol=1e-9)
    # the exact solution is a fixed point
    np.testing.assert_allclose(cp.gauss_seidel(exact, Gam, B, 10), exact, rtol=1e-12, atol=1e-12)
    # one iteration on a 2x2 system, written out by hand
    G2 = np.array([[4.0, 1.0], [1.0, 3.0]])
    b = np.array([[1.0, 2.0]])
    x0 = np.array([[0.5, -0.25]])
    x1 = (1.0 - 1.0 * -0.25) / 4.0
    x2 = (2.0 - 1.0 * x1) / 3.0
    np.testing.assert_allclose(cp.gauss_seidel(x0, G2, b, 1), [[x1, x2]], rtol=1e-15)
    # each GS iteration does not increase the quadratic 1/2 x G x^T - b x^T
    q = lambda X: 0.5 * np.sum((X @ Gam) * X) - np.sum(B * X)
    X = X0.copy()
    for _ in range(5):
        Xn = cp.gauss_seidel(X, Gam, B, 1)
        assert q(Xn) <= q(X) + 1e-12
        X = Xn


def test_als_mode_update_is_least_squares():
    rng = np.random.default_rng(10)
    dims, R = (4, 5, 3), 2
    Z = rng.standard_normal(dims)
    A = rand_factors(rng, dims, R)
    for n in range(3):
        Gam = cp.gamma(cp.grams(A), n)
        new = cp.solve_gamma(brute_mttkrp(Z, A, n), Gam)
        # numpy lstsq on the explicit design matrix built by loops
        others = [m for m in range(3) if m != n]
        rows = []
        ys = []
        for i in range(dims[n]):
            pass
        design = np.zeros((int(np.prod([dims[m] for m in others])), R))
        for k, idx in enumerate(itertools.product(*[range(dims[m]) for m in reversed(others)])):
            jdx = dict(zip(reversed(others), idx))
            for r in range(R):
                design[k, r] = np.prod([A[m][jdx[m], r] for m in others])
        target = np.zeros((design.shape[0], dims[n]))
        for k, idx in enumerate(itertools.product(*[range(dims[m]) for m in reversed(others)])):
            jdx = dict(zip(reversed(others), idx))
            for i in range(dims[n]):
                full_idx = [0, 0, 0]
                full_idx[n] = i
                for m in others:
                    full_idx[m] = jdx[m]
                target[k, i] = Z[tuple(full_idx)]
        ls = np.linalg.lstsq(design, target, rcond=None)[0].T
        np.testing.assert_allclose(new, ls, rtol=1e-10, atol=1e-12)
        del rows, ys


def test_als_update_zeroes_mode_gradient():
    rng = np.random.default_rng(11)
    dims, R = (3, 4, 3), 2
    Z = rng.standard_normal(dims)
    A = rand_factors(rng, dims, R)
    B = cp.als_sweep(Z, A, normalize_after=False)
    # after a full sweep the last mode's gradient is zero (it was just solved)
    h = 1e-6
    for i in range(dims[2]):
        for r in range(R):
            Ap = [a.copy() for a in B]
            Am = [a.copy() for a in B]
            Ap[2][i, r] += h
            Am[2][i, r] -= h
            fd = (brute_objective(Z, Ap) - brute_objective(Z, Am)) / (2 * h)
            assert abs(fd) < 1e-6


def test_normalize_and_sort():
    rng = np.random.default_rng(12)
    A = rand_factors(rng, (4, 5, 6), 3)
    A[0][:, 1] *= 100.0
    An = cp.normalize(A)
    np.testing.assert_allclose(cp.full(An), cp.full(A), rtol=1e-14, atol=1e-13)
    nr = np.array([np.linalg.norm(a, axis=0) for a in An])
    np.testing.assert_allclose(nr, np.tile(nr[0], (3, 1)), rtol=1e-14)
    lam = np.prod(np.array([np.linalg.norm(a, axis=0) for a in A]), axis=0) ** (1 / 3)
    np.testing.assert_allclose(nr[0], lam, rtol=1e-14)
    As, order = cp.sort_components(An)
    assert list(order) == list(np.argsort(-lam, kind="stable"))
    # a zero column leaves its component untouched
    A[1][:, 0] = 0.0
    An = cp.normalize(A)
    for n in range(3):
        np.testing.assert_array_equal(An[n][:, 0], A[n][:, 0])


def test_als_monotone_decrease():
    Z, _ = synth.collinear_tensor((10, 11, 12), 3, 0.9, 0.05, 0.02, seed=13)
    A = synth.uniform_start(Z.shape, 3, 13)
    f_prev = cp.objective(Z, A)
    nz2 = float(np.sum(Z ** 2))
    for _ in range(30):
        A = cp.als_sweep(Z, A)
        f = cp.objective(Z, A)
        assert f <= f_prev + 1e-13 * nz2
        f_prev = f


def test_exact_recovery_noise_free():
    dims, R = (20, 20, 20), 3
    Z, At = synth.collinear_tensor(dims, R, 0.5, 0.0, 0.0, seed=14)
    A0 = synth.uniform_start(dims, R, 14)
    A, hist = cp.als(Z, A0, max_sweeps=3000, fit_tol=0.0, g_tol=1e-13, record="fused")
    rel = np.sqrt(2 * cp.objective(Z, A)) / np.linalg.norm(Z)
    assert rel < 1e-12
    # factor congruence after permutation and sign matching
    for n in range(3):
        a = A[n] / np.linalg.norm(A[n], axis=0)
        t = At[n] / np.linalg.norm(At[n], axis=0)
        C = np.abs(a.T @ t)
        assert np.all(np.max(C, axis=1) > 1 - 1e-8)


def test_vanishing_gradient_at_convergence():
    Z, _ = synth.collinear_tensor((12, 13, 14), 3, 0.5, 0.01, 0.0, seed=15)
    A, hist = cp.als(Z, synth.uniform_start(Z.shape, 3, 15), max_sweeps=5000, fit_tol=0.0,
                     g_tol=1e-14, record="fused")
    G = cp.grams(A)
    phin = [np.linalg.norm(cp.phi(A, n)) for n in range(3)]
    for n in range(3):
        res = A[n] @ cp.gamma(G, n) - brute_mttkrp(Z, A, n) if Z.size < 3000 else \
            A[n] @ cp.gamma(G, n) - cp.mttkrp(Z, A, n)
        assert np.linalg.norm(res) / (np.linalg.norm(Z) * phin[n]) < 1e-12


def test_fused_objective_tracks_direct_in_als():
    Z, _ = synth.collinear_tensor((9, 10, 11), 3, 0.5, 0.05, 0.0, seed=16)
    A0 = synth.uniform_start(Z.shape, 3, 16)
    _, h1 = cp.als(Z, A0, max_sweeps=15, fit_tol=0.0, record="fused", sort_at_end=False)
    _, h2 = cp.als(Z, A0, max_sweeps=15, fit_tol=0.0, record="direct", sort_at_end=False)
    np.testing.assert_allclose(h1["f"], h2["f"], rtol=1e-10)

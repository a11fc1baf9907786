"""Pins of the multilevel oracle (Sections 4-6) against brute force, closed forms
and the exactness statements of the paper."""
import itertools

import numpy as np
import pytest

from oracle import amg, cp
from paper_1111_6091_amd import synth


def brute_restrict(Z, Rh):
    """Zc[j...] = sum_i Z[i...] prod_n Rh_n[j_n, i_n] by explicit loops."""
    dims = Z.shape
    cdims = [r.shape[0] if r is not None else d for r, d in zip(Rh, dims)]
    out = np.zeros(cdims)
    for jdx in itertools.product(*[range(d) for d in cdims]):
        s = 0.0
        for idx in itertools.product(*[range(d) for d in dims]):
            p = Z[idx]
            for n in range(len(dims)):
                if Rh[n] is None:
                    if idx[n] != jdx[n]:
                        p = 0.0
                        break
                else:
                    p *= Rh[n][jdx[n], idx[n]]
            s += p
        out[jdx] = s
    return out


def random_weights(rng, I):
    w = np.zeros((I, 2))
    for i in range(1, I, 2):
        w[i] = rng.uniform(0.1, 0.9, 2)
        if i + 1 >= I:
            w[i, 1] = 0.0
    return w


@pytest.mark.parametrize("I", [5, 6, 7, 20, 128])
def test_interpolation_structure(I):
    rng = np.random.default_rng(0)
    w = random_weights(rng, I)
    P = amg.interp_from_weights(I, w)
    Ic = amg.coarse_size(I)
    assert P.shape == (I, Ic)
    for i in range(0, I, 2):                       # coarse rows are injections
        assert P[i, i // 2] == 1.0 and np.count_nonzero(P[i]) == 1
    for i in range(1, I, 2):                       # fine rows use alpha(i-1), alpha(i+1)
        nz = set(np.nonzero(P[i])[0])
        assert nz <= {(i - 1) // 2, (i + 1) // 2}
        if i + 1 >= I:
            assert nz == {(i - 1) // 2}
    B, L, Phat = amg.transfer(P)
    # B = P^T P is tridiagonal, so L is lower bidiagonal
    assert np.allclose(np.triu(B, 2), 0) and np.allclose(np.tril(B, -2), 0)
    assert np.allclose(np.tril(L, -2), 0)
    # P^ has orthonormal columns: P^^T P^ = L^{-1} B L^{-T} = I
    np.testing.assert_allclose(Phat.T @ Phat, np.eye(Ic), atol=1e-13)
    # closed forms of the prolongation: P^ L^T Ac = P Ac, R^ P^ = I
    Ac = rng.standard_normal((Ic, 3))
    np.testing.assert_allclose(Phat @ (L.T @ Ac), P @ Ac, rtol=1e-12, atol=1e-12)
    # P^ spans the same range as P
    np.testing.assert_allclose(Phat @ (Phat.T @ P), P, atol=1e-12)


def test_restriction_brute_force_and_identity():
    rng = np.random.default_rng(1)
    dims = (5, 4, 3)
    Z = rng.standard_normal(dims)
    Ph = [amg.transfer(amg.interp_from_weights(d, random_weights(rng, d)))[2] for d in dims]
    Rh = [p.T for p in Ph]
    np.testing.assert_allclose(amg.restrict_tensor(Z, Rh), brute_restrict(Z, Rh), rtol=1e-12, atol=1e-12)
    Rh2 = [Rh[0], None, Rh[2]]
    np.testing.assert_allclose(amg.restrict_tensor(Z, Rh2), brute_restrict(Z, Rh2), rtol=1e-12, atol=1e-12)
    # identity restriction returns Z bit for bit
    np.testing.assert_array_equal(amg.restrict_tensor(Z, [None, None, None]), Z)


def test_coarse_tensor_closed_form_and_pythagoras():
    """If Z = [[P A_c]] then Z^c = [[L^T A_c]] exactly (Sec. 4.1), and
    f(P^ A^) = f^_c(A^) + 1/2 (||Z||^2 - ||Z^c||^2) for any coarse A^."""
    rng = np.random.default_rng(2)
    dims, R = (9, 8, 7), 2
    trip = [amg.transfer(amg.interp_from_weights(d, random_weights(rng, d))) for d in dims]
    Ps = [amg.interp_from_weights(d, random_weights(np.random.default_rng(2 + k), d))
          for k, d in enumerate(dims)]
    trip = [amg.transfer(P) for P in Ps]
    Ac = [rng.standard_normal((amg.coarse_size(d), R)) for d in dims]
    Z = cp.full([P @ a for P, a in zip(Ps, Ac)])
    Zc = amg.restrict_tensor(Z, [t[2].T for t in trip])
    np.testing.assert_allclose(Zc, cp.full([t[1].T @ a for t, a in zip(trip, Ac)]),
                               rtol=1e-11, atol=1e-11)
    Zr = rng.standard_normal(dims)
    Zrc = amg.restrict_tensor(Zr, [t[2].T for t in trip])
    Ahat = [rng.standard_normal((amg.coarse_size(d), R)) for d in dims]
    lhs = cp.objective(Zr, amg.prolong([t[2] for t in trip], Ahat))
    rhs = cp.objective(Zrc, Ahat) + 0.5 * (np.sum(Zr ** 2) - np.sum(Zrc ** 2))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_ls_weights_exact_cases():
    rng = np.random.default_rng(3)
    I = 9
    # vectors that are exactly linearly interpolated are reproduced: weights (1/2, 1/2)
    U = np.zeros((I, 4))
    for k in range(4):
        U[0::2, k] = rng.standard_normal(amg.coarse_size(I))
        U[1:I - 1:2, k] = 0.5 * (U[0:I - 2:2, k] + U[2::2, k])
    w = amg.ls_interp_weights(U, np.ones(4))
    np.testing.assert_allclose(w[1:I - 1:2], 0.5, rtol=1e-12)
    # one vector, single-neighbour right endpoint: exact fit
    I = 8
    u = rng.standard_normal((I, 1))
    w = amg.ls_interp_weights(np.hstack([u, rng.standard_normal((I, 2))]), [1.0, 1.0, 1.0])
    w1 = amg.ls_interp_weights(u, [1.0])
    assert w1[I - 1, 0] * u[I - 2, 0] == pytest.approx(u[I - 1, 0], rel=1e-12)
    # a heavily weighted vector is fitted (nearly) exactly
    U = rng.standard_normal((I, 3))
    w = amg.ls_interp_weights(U, [1e12, 1.0, 1.0])
    P = amg.interp_from_weights(I, w)
    inj = U[0::2, 0]
    assert np.linalg.norm(P @ inj - U[:, 0]) > 0   # 2 weights cannot fit 3 vectors exactly
    # two independent vectors make the two-neighbour fits exact (the single-
    # neighbour right endpoint of an even-length mode is overdetermined)
    U2 = rng.standard_normal((I, 2))
    P2 = amg.interp_from_weights(I, amg.ls_interp_weights(U2, [1.0, 1.0]))
    np.testing.assert_allclose((P2 @ U2[0::2])[:-1], U2[:-1], rtol=1e-10, atol=1e-12)


def test_block_weight_definition():
    rng = np.random.default_rng(4)
    Z = rng.standard_normal((4, 5, 6))
    A = [rng.standard_normal((d, 2)) for d in (4, 5, 6)]
    G = cp.gradient(Z, A)
    for n in range(3):
        assert amg.block_weight(Z, A, n) == pytest.approx(np.sum(A[n] ** 2) / np.sum(G[n] ** 2), rel=1e-12)


def test_block_weight_floor_after_an_als_sweep():
    """After an ALS sweep the last mode's gradient vanishes identically (its
    computed norm is rounding noise): the weight takes the floor
    ||A||^2 / (1e-8 ||M||)^2 whatever the rounding; the other modes keep their
    true gradients."""
    from paper_1111_6091_amd import synth
    Z, _ = synth.collinear_tensor((9, 8, 7), 2, 0.5, 0.05, 0.0, seed=3)
    A = cp.als_sweep(Z, synth.uniform_start((9, 8, 7), 2, 3))
    G = cp.gradient(Z, A)
    M2 = cp.mttkrp(Z, A, 2)
    assert np.linalg.norm(G[2]) < 1e-12 * np.linalg.norm(M2)
    w2 = amg.block_weight(Z, A, 2)
    assert w2 == pytest.approx(np.sum(A[2] ** 2) / (amg.GRAD_FLOOR ** 2 * np.sum(M2 ** 2)), rel=1e-12)
    for n in (0, 1):
        assert np.linalg.norm(G[n]) > 1e-6 * np.linalg.norm(cp.mttkrp(Z, A, n))
        assert amg.block_weight(Z, A, n) == pytest.approx(np.sum(A[n] ** 2) / np.sum(G[n] ** 2), rel=1e-12)


def test_fas_operator_is_gradient():
    """H^(n) of eq. (23) is the partial derivative of f (compare eq. (6))."""
    rng = np.random.default_rng(5)
    Z = rng.standard_normal((3, 4, 2))
    A = [rng.standard_normal((d, 2)) for d in (3, 4, 2)]
    H = amg.fas_H(Z, A)
    h = 1e-6
    for n in range(3):
        for i in range(A[n].shape[0]):
            for r in range(2):
                Ap = [a.copy() for a in A]
                Am = [a.copy() for a in A]
                Ap[n][i, r] += h
                Am[n][i, r] -= h
                fd = (cp.objective(Z, Ap) - cp.objective(Z, Am)) / (2 * h)
                assert H[n][i, r] == pytest.approx(fd, rel=1e-6, abs=1e-7)


def test_bngs_with_rhs_decreases_phi():
    """BNGS on H(A) = F is block coordinate descent on phi(A) = f(A) - sum_n <F^(n), A^(n)>."""
    Z, _ = synth.collinear_tensor((8, 9, 10), 3, 0.7, 0.05, 0.0, seed=6)
    rng = np.random.default_rng(6)
    A = synth.uniform_start(Z.shape, 3, 6)
    F = [0.3 * rng.standard_normal(a.shape) for a in A]
    phi = lambda A: cp.objective(Z, A) - sum(float(np.sum(f * a)) for f, a in zip(F, A))
    p = phi(A)
    for _ in range(10):
        A = amg.bngs(Z, A, F, gs_iters=10)
        pn = phi(A)
        assert pn <= p + 1e-12 * abs(p)
        p = pn


def _two_level(Z, R, seed=7):
    rng = np.random.default_rng(seed)
    w = [random_weights(rng, d) for d in Z.shape]
    return amg.hierarchy_from_weights(Z, [w], [amg.coarse_size(d) for d in Z.shape])


def test_fas_fixed_point():
    """A converged solution is a fixed point of the CP-FAS V-cycle (Sec. 5.2)."""
    Z, _ = synth.collinear_tensor((12, 12, 12), 3, 0.5, 0.01, 0.0, seed=8)
    A, h = cp.als(Z, synth.uniform_start(Z.shape, 3, 8), max_sweeps=5000, fit_tol=0.0, g_tol=1e-13)
    levels = _two_level(Z, 3)
    A1 = amg.fas_vcycle(levels, amg.zeros_like_factors(A), A, nu1=1, nu2=1, nuc=50)
    T0, T1 = cp.full(A), cp.full(A1)
    assert np.linalg.norm(T1 - T0) / np.linalg.norm(T0) < 1e-10


def test_fas_identity_transfers_equal_plain_bngs():
    """With P^ = I on every mode the 2-level V-cycle equals nu1 + nuc + nu2 BNGS sweeps."""
    Z, _ = synth.collinear_tensor((7, 8, 9), 2, 0.6, 0.05, 0.0, seed=9)
    A0 = synth.uniform_start(Z.shape, 2, 9)
    eye = [np.eye(d) for d in Z.shape]
    levels = [amg.Level(Z, eye), amg.Level(amg.restrict_tensor(Z, [e.T for e in eye]), [None] * 3)]
    A1 = amg.fas_vcycle(levels, amg.zeros_like_factors(A0), A0, nu1=1, nu2=1, nuc=3)
    A2 = A0
    for _ in range(5):
        A2 = amg.bngs(Z, A2, amg.zeros_like_factors(A0), normalize_after=False)
    np.testing.assert_allclose(cp.full(A1), cp.full(A2), rtol=1e-9, atol=1e-11)


def test_fas_literal_and_tau_rules_agree_when_all_modes_coarsen():
    Z, _ = synth.collinear_tensor((10, 10, 10), 2, 0.5, 0.02, 0.0, seed=10)
    A0 = synth.uniform_start(Z.shape, 2, 10)
    levels = _two_level(Z, 2, seed=10)
    a = amg.fas_vcycle(levels, amg.zeros_like_factors(A0), A0, ic_rule="tau", nuc=5)
    b = amg.fas_vcycle(levels, amg.zeros_like_factors(A0), A0, ic_rule="literal", nuc=5)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_fas_uneven_modes_tau_rule_keeps_fixed_point():
    """Mode 3 is not coarsened (I_c' nonempty); the tau rule keeps the fixed point."""
    Z, _ = synth.collinear_tensor((12, 12, 4), 2, 0.5, 0.01, 0.0, seed=11)
    A, _ = cp.als(Z, synth.uniform_start(Z.shape, 2, 11), max_sweeps=5000, fit_tol=0.0, g_tol=1e-13)
    rng = np.random.default_rng(11)
    w = [random_weights(rng, 12), random_weights(rng, 12), None]
    levels = amg.hierarchy_from_weights(Z, [w], [6, 6, 4])
    assert levels[0].Phat[2] is None
    A1 = amg.fas_vcycle(levels, amg.zeros_like_factors(A), A, ic_rule="tau")
    assert np.linalg.norm(cp.full(A1) - cp.full(A)) / np.linalg.norm(cp.full(A)) < 1e-10


def test_setup_and_solve_phase_reduce_g():
    Z, _ = synth.collinear_tensor((16, 16, 16), 2, 0.5, 0.01, 0.0, seed=12)
    A0 = synth.uniform_start(Z.shape, 2, 12)
    tfms = [synth.uniform_start(Z.shape, 2, 100 + t) for t in range(2)]
    coarsest = [4, 4, 4]
    g0 = cp.grad_norm(Z, A0)
    A, tfms, levels, hist = amg.setup_phase(Z, A0, tfms, coarsest, nu1=2, nu2=2, nuc=20)
    assert len(levels) == amg.n_levels(Z.shape, coarsest) == 3
    assert hist[-1] < g0
    for lev in levels[:-1]:
        for p in lev.Phat:
            np.testing.assert_allclose(p.T @ p, np.eye(p.shape[1]), atol=1e-12)
    A2, levels2, h2 = amg.solve_phase(Z, A, levels, tfms, coarsest, max_cycles=3, nuc=10)
    assert h2[-1] < hist[-1]
    # FMG cycle runs over the same hierarchy and returns finest-level factors
    Af = amg.fmg_cycle(levels, synth.uniform_start(levels[-1].dims, 2, 13), nu=20, nuc=10)
    assert [a.shape for a in Af] == [a.shape for a in A0]

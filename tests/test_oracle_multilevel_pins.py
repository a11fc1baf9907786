"""Pins of the multilevel oracle parts that drive whole cycles (Algorithms 1-3,
Section 6.1), each chosen so that one plausible mistake in the function fails it:

* CP-FAS V-cycle (Alg. 2) at three levels: the fixed point (a converged ALS
  solution is left in place, which needs the coarse right-hand side eq. (27) to
  be passed down correctly at depth two and normalization to stay on the top
  level) and identity transfers (the cycle is then exactly the BNGS sweeps it
  schedules: the level recursion and the sweep counts).
* FMG-CP-FAS (Alg. 3): exact reproduction of a tensor that lies in the range of
  the interpolation (prolongation direction and order of the steps), and with
  identity transfers the ALS iterations of the coarsest level followed by the
  V-cycles' sweeps (the level loop).
* Least-squares interpolation (Sec. 4.4, eqs. (19)-(20)): exactly interpolable
  TFMs and BFMs are reproduced; the boot block enters only when asked for.
* Setup V-cycle (Alg. 1): the first cycle fits the TFMs only, later cycles also
  the BFMs (a block with a vanishing gradient dominates the fit, eq. (20)).
* Down-sweep of the Section 6.1 rebuild: the boot factors enter the fit as given
  (neither relaxed nor modified).
* Setup-phase stopping (eq. (32), Section 6.1): checked only once three cycles
  have completed, against the previous cycle, at most five cycles.
* Solve-phase stagnation (Section 6.1): checked only after five cycles; the
  stagnating iterate is discarded and the operators rebuilt from the previous
  one, at most once.
"""
import numpy as np
import pytest

from oracle import amg, cp
from paper_1111_6091_amd import synth


def random_weights(rng, I):
    w = np.zeros((I, 2))
    for i in range(1, I, 2):
        w[i] = rng.uniform(0.1, 0.9, 2)
        if i + 1 >= I:
            w[i, 1] = 0.0
    return w


def interpolable(rng, I, R, w):
    """I x R matrix whose columns are exactly P(w) times coarse vectors."""
    return amg.interp_from_weights(I, w) @ rng.standard_normal((amg.coarse_size(I), R))


def rel_change(A, B):
    TA, TB = cp.full(A), cp.full(B)
    return np.linalg.norm(TB - TA) / np.linalg.norm(TA)


# ---------------------------------------------------------------------------
# Algorithm 2 at three levels
# ---------------------------------------------------------------------------
def test_fas_three_level_fixed_point():
    Z, _ = synth.collinear_tensor((16, 16, 16), 3, 0.5, 0.01, 0.0, seed=21)
    A, _ = cp.als(Z, synth.uniform_start(Z.shape, 3, 21), max_sweeps=5000, fit_tol=0.0, g_tol=1e-13)
    assert cp.grad_norm(Z, A) < 1e-13
    rng = np.random.default_rng(21)
    w0 = [random_weights(rng, 16) for _ in range(3)]
    w1 = [random_weights(rng, 8) for _ in range(3)]
    levels = amg.hierarchy_from_weights(Z, [w0, w1], [4, 4, 4])
    assert len(levels) == 3 and levels[1].dims == (8, 8, 8) and levels[2].dims == (4, 4, 4)
    A1 = amg.fas_vcycle(levels, amg.zeros_like_factors(A), A, nu1=1, nu2=1, nuc=50)
    assert rel_change(A, A1) < 1e-10


def test_fas_three_level_fixed_point_detects_a_wrong_depth_two_rhs(monkeypatch):
    """Planted mistake (oracle, CPU): the coarsest level (depth two) solved with
    F = 0 instead of its coarse right-hand side.  The fixed-point pin above must
    then fail."""
    Z, _ = synth.collinear_tensor((16, 16, 16), 3, 0.5, 0.01, 0.0, seed=21)
    A, _ = cp.als(Z, synth.uniform_start(Z.shape, 3, 21), max_sweeps=5000, fit_tol=0.0, g_tol=1e-13)
    rng = np.random.default_rng(21)
    w0 = [random_weights(rng, 16) for _ in range(3)]
    w1 = [random_weights(rng, 8) for _ in range(3)]
    levels = amg.hierarchy_from_weights(Z, [w0, w1], [4, 4, 4])
    real = amg.fas_vcycle

    def broken(levels, F, A, l=0, *args, **kw):
        return real(levels, amg.zeros_like_factors(A) if l >= 2 else F, A, l, *args, **kw)

    monkeypatch.setattr(amg, "fas_vcycle", broken)
    A1 = amg.fas_vcycle(levels, amg.zeros_like_factors(A), A, nu1=1, nu2=1, nuc=50)
    assert rel_change(A, A1) > 1e-6


@pytest.mark.parametrize("nu1,nu2,nuc", [(1, 1, 3), (2, 1, 2)])
def test_fas_three_level_identity_transfers_are_plain_bngs(nu1, nu2, nuc):
    """P^ = I on every mode of both coarsenings: F_c = F on every level, so one
    V-cycle is exactly 2 nu1 + nuc + 2 nu2 BNGS sweeps (normalization on the top
    level does not change [[A]]: Gauss-Seidel is invariant under the diagonal
    rescaling, Section 5.2)."""
    Z, _ = synth.collinear_tensor((7, 8, 9), 2, 0.6, 0.05, 0.0, seed=22)
    A0 = synth.uniform_start(Z.shape, 2, 22)
    eye = [np.eye(d) for d in Z.shape]
    levels = [amg.Level(Z, eye), amg.Level(Z.copy(), eye), amg.Level(Z.copy(), [None] * 3)]
    A1 = amg.fas_vcycle(levels, amg.zeros_like_factors(A0), A0, nu1=nu1, nu2=nu2, nuc=nuc)
    A2 = A0
    for _ in range(2 * nu1 + nuc + 2 * nu2):
        A2 = amg.bngs(Z, A2, amg.zeros_like_factors(A0), normalize_after=False)
    assert rel_change(A2, A1) < 1e-9
    # one sweep more or less is far away
    A3 = amg.bngs(Z, A2, amg.zeros_like_factors(A0), normalize_after=False)
    assert rel_change(A3, A1) > 1e-6


# ---------------------------------------------------------------------------
# Algorithm 3
# ---------------------------------------------------------------------------
def test_fmg_reproduces_a_tensor_in_the_range_of_p():
    """Z = [[P A_c]] and the exact coarse solution L^T A_c (Sec. 4.1): the
    coarsest ALS keeps it, P^ L^T A_c = P A_c reproduces Z, and the fine
    V-cycle (F = 0) leaves an exact solution in place."""
    rng = np.random.default_rng(23)
    dims, R = (10, 12, 9), 2
    ws = [random_weights(rng, d) for d in dims]
    Ps = [amg.interp_from_weights(d, w) for d, w in zip(dims, ws)]
    Ls = [amg.transfer(P)[1] for P in Ps]
    Ac = [rng.standard_normal((amg.coarse_size(d), R)) for d in dims]
    Z = cp.full([P @ a for P, a in zip(Ps, Ac)])
    levels = amg.hierarchy_from_weights(Z, [ws], [amg.coarse_size(d) for d in dims])
    assert len(levels) == 2
    Af = amg.fmg_cycle(levels, [L.T @ a for L, a in zip(Ls, Ac)], nu=5, nuc=5)
    assert [a.shape for a in Af] == [(d, R) for d in dims]
    assert np.linalg.norm(cp.full(Af) - Z) / np.linalg.norm(Z) < 1e-10
    # prolonging with P instead of P^ (a plausible mistake) does not reproduce Z
    wrong = [P @ (L.T @ a) for P, L, a in zip(Ps, Ls, Ac)]
    assert np.linalg.norm(cp.full(wrong) - Z) / np.linalg.norm(Z) > 1e-3


def test_fmg_identity_transfers_are_als_then_vcycle_sweeps():
    """Three levels with P^ = I: nu ALS iterations on the coarsest level, then the
    level-1 V-cycle (nu1 + nuc + nu2 BNGS sweeps) and the level-0 V-cycle
    (2 nu1 + nuc + 2 nu2)."""
    Z, _ = synth.collinear_tensor((7, 8, 9), 2, 0.6, 0.05, 0.0, seed=24)
    A0 = synth.uniform_start(Z.shape, 2, 24)
    eye = [np.eye(d) for d in Z.shape]
    levels = [amg.Level(Z, eye), amg.Level(Z.copy(), eye), amg.Level(Z.copy(), [None] * 3)]
    nu, nu1, nu2, nuc = 4, 1, 1, 2
    Af = amg.fmg_cycle(levels, A0, nu=nu, nu1=nu1, nu2=nu2, nuc=nuc)
    A = A0
    for _ in range(nu):
        A = cp.als_sweep(Z, A)
    for _ in range((nu1 + nuc + nu2) + (2 * nu1 + nuc + 2 * nu2)):
        A = amg.bngs(Z, A, amg.zeros_like_factors(A0), normalize_after=False)
    assert rel_change(A, Af) < 1e-9


# ---------------------------------------------------------------------------
# Section 4.4: least-squares interpolation
# ---------------------------------------------------------------------------
def test_build_interp_reproduces_exactly_interpolable_blocks():
    rng = np.random.default_rng(25)
    dims, R, n = (11, 6, 5), 3, 0
    Z = rng.standard_normal(dims)
    wstar = random_weights(rng, dims[n])

    def block(interp):
        return [interpolable(rng, d, R, wstar) if (m == n and interp) else rng.uniform(0, 1, (d, R))
                for m, d in enumerate(dims)]

    tfms = [block(True), block(True)]
    good_bfm, bad_bfm = block(True), block(False)
    fine = slice(1, dims[n], 2)
    for use_bfm in (False, True):
        w = amg.build_interp(Z, tfms, good_bfm, n, use_bfm)
        np.testing.assert_allclose(w[fine], wstar[fine], rtol=1e-10, atol=1e-12)
    # a boot block that is not interpolable enters only when asked for
    np.testing.assert_allclose(amg.build_interp(Z, tfms, bad_bfm, n, False)[fine], wstar[fine],
                               rtol=1e-10, atol=1e-12)
    assert np.max(np.abs(amg.build_interp(Z, tfms, bad_bfm, n, True)[fine] - wstar[fine])) > 1e-6


def _stationary_interpolable_problem(seed, dims=(12, 12, 12), R=2, noise=0.1):
    """Z = [[B]] + E with B exactly interpolable and E orthogonal to every
    Z_(n) Phi^(n)(B) direction, so that every G^(n)(B) vanishes (eq. (6)): B is
    a stationary point, kept by ALS sweeps, while iterates from other starts are
    generic (E has components outside the range of B)."""
    rng = np.random.default_rng(seed)
    ws = [random_weights(rng, d) for d in dims]
    B = [interpolable(rng, d, R, w) for d, w in zip(dims, ws)]
    T = cp.full(B)
    rows = []
    for n, d in enumerate(dims):
        Phi = cp.phi(B, n)
        for i in range(d):
            for r in range(R):
                K = np.zeros((d, Phi.shape[0]))
                K[i] = Phi[:, r]
                rows.append(cp.fold(K, n, dims).ravel())
    C = np.array(rows)
    E = rng.standard_normal(T.size)
    E = E - C.T @ np.linalg.lstsq(C @ C.T, C @ E, rcond=None)[0]
    E = E.reshape(dims)
    Z = T + noise * np.linalg.norm(T) * E / np.linalg.norm(E)
    G = cp.gradient(Z, B)
    assert max(np.linalg.norm(g) for g in G) < 1e-10 * np.linalg.norm(Z) * max(np.linalg.norm(b) for b in B)
    return Z, B, ws


def test_setup_vcycle_fits_tfms_first_then_bfms():
    """Alg. 1 line 3: the first cycle builds P from the TFMs only; later cycles add
    the BFMs.  Here the BFMs are an exactly interpolable stationary point, so
    their gradient vanishes, their weight (eq. (20)) dominates and the fit returns
    their interpolation weights; the relaxed TFMs are generic."""
    Z, B, ws = _stationary_interpolable_problem(26)
    dims = Z.shape
    tfms = [synth.uniform_start(dims, 2, 260 + t) for t in range(2)]
    fine = slice(1, dims[0], 2)
    for first in (True, False):
        _, _, lv = amg.mult_vcycle(Z, [b.copy() for b in B], tfms, [6, 6, 6], first_cycle=first,
                                   nu1=1, nu2=1, nuc=5)
        assert len(lv) == 2
        dev = np.max(np.abs(lv[0].weights[0][fine] - ws[0][fine]))
        if first:
            assert dev > 1e-3, dev
        else:
            assert dev < 1e-8, dev


def test_down_sweep_uses_the_boot_factors_as_given():
    """Section 6.1: the rebuild does not update the boot factors.  Boot factors
    whose mode-0 factor is exactly interpolable and optimal for the other two
    (G^(0) = 0, eq. (6)) without being a solution: the fit of mode 0 returns
    their weights exactly; relaxing them first (the mistake) would not."""
    rng = np.random.default_rng(27)
    dims, R = (12, 10, 8), 2
    w0 = random_weights(rng, dims[0])
    B = [interpolable(rng, dims[0], R, w0), rng.standard_normal((dims[1], R)),
         rng.standard_normal((dims[2], R))]
    T = cp.full(B)
    # noise whose mode-0 unfolding is orthogonal to Phi^(0): G^(0)(B) = 0
    Phi = cp.phi(B, 0)
    E = rng.standard_normal((dims[0], Phi.shape[0]))
    E = E - (E @ Phi) @ np.linalg.solve(Phi.T @ Phi, Phi.T)
    E = cp.fold(E, 0, dims)
    Z = T + 0.1 * np.linalg.norm(T) * E / np.linalg.norm(E)
    G = cp.gradient(Z, B)
    assert np.linalg.norm(G[0]) < 1e-10 * np.linalg.norm(B[0]) * np.linalg.norm(Z)
    assert np.linalg.norm(G[1]) > 1e-3
    tfms = [synth.uniform_start(dims, R, 270 + t) for t in range(2)]
    B_in = [b.copy() for b in B]
    tf_in = [[a.copy() for a in t] for t in tfms]
    levels, fine_tfms = amg.down_sweep(Z, B_in, tf_in, [6, 5, 4], nu1=2)
    for a, b in zip(B_in, B):                      # inputs are not modified
        np.testing.assert_array_equal(a, b)
    for t_in, t in zip(tf_in, tfms):
        for a, b in zip(t_in, t):
            np.testing.assert_array_equal(a, b)
    fine = slice(1, dims[0], 2)
    assert np.max(np.abs(levels[0].weights[0][fine] - w0[fine])) < 1e-8
    # the mistake: boot factors relaxed as the TFMs are
    Br = B
    for _ in range(2):
        Br = cp.als_sweep(Z, Br)
    w_bad = amg.build_interp(Z, fine_tfms, Br, 0, use_bfm=True)
    assert np.max(np.abs(w_bad[fine] - w0[fine])) > 1e-6


# ---------------------------------------------------------------------------
# Section 6.1 driver rules
# ---------------------------------------------------------------------------
def _marker(k):
    return [np.array([[float(k)]])]


def test_setup_phase_stagnation_rule(monkeypatch):
    """eq. (32) with eps = 0.1: checked after cycles 3, 4 and 5 against the
    previous cycle; at most five cycles."""
    def run(gseq):
        state = {"k": 0}

        def cycle(Z, A, tfms, coarsest, first_cycle, **kw):
            state["k"] += 1
            assert first_cycle == (state["k"] == 1)
            return _marker(state["k"]), tfms, ["levels", state["k"]]

        monkeypatch.setattr(amg, "mult_vcycle", cycle)
        monkeypatch.setattr(amg.cp, "grad_norm", lambda Z, A: gseq[int(A[0][0, 0])])
        A, tfms, levels, hist = amg.setup_phase(None, _marker(0), [], None)
        return state["k"], hist, levels

    # stagnating from the first cycle: not checked before three cycles completed
    k, hist, levels = run([1.0, 0.99, 0.98, 0.97, 0.5, 0.1])
    assert k == 3 and hist == [0.99, 0.98, 0.97] and levels == ["levels", 3]
    # fast decrease: five cycles
    k, hist, _ = run([1.0, 0.5, 0.25, 0.12, 0.06, 0.03, 0.01])
    assert k == 5
    # compared with the previous cycle (0.2 > 0.9 * 0.25 is false; 0.19 > 0.9 * 0.2 is true)
    k, _, _ = run([1.0, 0.5, 0.25, 0.2, 0.19, 0.01])
    assert k == 4


def test_solve_phase_stagnation_rebuild(monkeypatch):
    """Section 6.1: from cycle 6 on, g_new >= g_old discards the new iterate and
    rebuilds the operators once by a down-sweep with the previous iterate as boot
    factors; later stagnation is ignored; stop when g < tau."""
    g = {0: 1.0, 1: 0.5, 2: 0.4, 3: 0.3, 4: 0.2, 5: 0.25, 6: 0.3, 7: 0.05, 8: 0.06, 9: 1e-11}
    seen = {"v": 0, "levels": [], "down": []}

    def vcycle(levels, F, A, **kw):
        seen["v"] += 1
        seen["levels"].append(levels)
        return _marker(seen["v"])

    def down(Z, A, tfms, coarsest, nu1=5, use_bfm=True):
        seen["down"].append((int(A[0][0, 0]), nu1))
        return "rebuilt", tfms

    monkeypatch.setattr(amg, "fas_vcycle", vcycle)
    monkeypatch.setattr(amg, "down_sweep", down)
    monkeypatch.setattr(amg.cp, "grad_norm", lambda Z, A: g[int(A[0][0, 0])])
    A, levels, hist = amg.solve_phase(None, _marker(0), "initial", [], None, tau=1e-10)
    # cycle 5 (0.25 >= 0.2) is not checked; cycle 6 (0.3 >= 0.25) rebuilds from iterate 5
    assert seen["down"] == [(5, 5)]
    assert seen["levels"][:6] == ["initial"] * 6 and seen["levels"][6:] == ["rebuilt"] * 3
    assert int(A[0][0, 0]) == 9 and levels == "rebuilt"
    assert hist == [0.5, 0.4, 0.3, 0.2, 0.25, 0.05, 0.06, 1e-11]

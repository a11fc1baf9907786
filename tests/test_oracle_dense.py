"""The dense test problem of Section 6.3 and the 'Multilevel + FMG' combination
of Section 6.1 in the oracle: the closed-form tensor, the coarsening thresholds
read off Table 4's level counts, the order of the combination's stages, and
convergence on a small instance against standalone ALS."""
import json
import os

import numpy as np
import pytest

from oracle import amg, cp
from paper_1111_6091_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_dense_tensor_closed_form():
    """Entries (i^2 + j^2 + k^2)^(-1/2) with 1-based indices, symmetric in the
    three modes, Fortran (mode 1 fastest) layout."""
    s = 7
    Z = synth.dense_ijk(s)
    assert Z.shape == (s, s, s) and Z.flags.f_contiguous
    assert Z[0, 0, 0] == pytest.approx(1.0 / np.sqrt(3.0), rel=1e-15)
    assert Z[s - 1, s - 1, s - 1] == pytest.approx(1.0 / (s * np.sqrt(3.0)), rel=1e-15)
    # (1, 2, 2): 1 + 4 + 4 = 9
    assert Z[0, 1, 1] == pytest.approx(1.0 / 3.0, rel=1e-15)
    # (2, 3, 6): 4 + 9 + 36 = 49 in every order of the modes
    for idx in [(1, 2, 5), (5, 1, 2), (2, 5, 1), (1, 5, 2)]:
        assert Z[idx] == pytest.approx(1.0 / 7.0, rel=1e-15)
    for perm in [(1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)]:
        assert np.array_equal(Z, np.transpose(Z, perm))
    # linear offset of (i, j, k) is i + s j + s^2 k
    flat = Z.ravel(order="K")
    assert flat[1 + s * 2 + s * s * 5] == Z[1, 2, 5]


def test_coarsening_threshold_reproduces_table4_levels():
    """I_{n,coarsest} = 2R (modes coarsened while larger, odd points coarse) gives
    the level count Table 4 lists for each of its twelve tests."""
    with open(os.path.join(HERE, "golden", "table4_dense_levels.json")) as f:
        rows = json.load(f)["tests"]
    assert len(rows) == 12
    for row in rows:
        s, R = row["s"], row["R"]
        assert synth.DENSE_TESTS[row["test"]] == (s, R)
        coarsest = synth.dense_case(s, R)["coarsest"] if s <= 50 else [2 * R] * 3
        assert amg.n_levels((s, s, s), coarsest) == row["levs"], row


def _marker(k):
    return [np.array([[float(k)]])]


def test_multilevel_fmg_stage_order(monkeypatch):
    """Section 6.1: setup cycles; one FMG cycle over the setup's levels from the
    coarsest-level start; its result becomes the boot factors of one down-sweep
    that rebuilds the operators from the setup's test blocks (and relaxes them);
    the solve cycles start from the FMG result on the rebuilt levels, with the
    relaxed test blocks for a later rebuild."""
    calls = []

    def setup(Z, A0, tfms0, coarsest, **kw):
        calls.append(("setup", int(A0[0][0, 0]), tfms0))
        return _marker(1), "tfms_after_setup", "setup_levels", [0.3, 0.2, 0.19]

    def fmg(levels, start, nu=100, **kw):
        calls.append(("fmg", levels, int(start[0][0, 0]), nu))
        return _marker(2)

    def down(Z, A, tfms, coarsest, nu1=5, use_bfm=True):
        calls.append(("down", int(A[0][0, 0]), tfms, nu1))
        return "rebuilt_levels", "tfms_after_down"

    def solve(Z, A, levels, tfms, coarsest, tau=1e-10, max_cycles=500, stagnation_after=5,
              nu1_setup=5, info=None, **fas):
        calls.append(("solve", int(A[0][0, 0]), levels, tfms, tau, fas))
        info["rebuilt"] = False
        return _marker(3), levels, [1e-3, 1e-7, 1e-11]

    monkeypatch.setattr(amg, "setup_phase", setup)
    monkeypatch.setattr(amg, "fmg_cycle", fmg)
    monkeypatch.setattr(amg, "down_sweep", down)
    monkeypatch.setattr(amg, "solve_phase", solve)
    monkeypatch.setattr(amg.cp, "grad_norm", lambda Z, A: 0.5)
    A, info = amg.multilevel_fmg(None, _marker(0), "tfms0", None, _marker(9), tau=1e-10,
                                 fmg_nu=100, fas=dict(nu1=1))
    assert calls == [
        ("setup", 0, "tfms0"),
        ("fmg", "setup_levels", 9, 100),
        ("down", 2, "tfms_after_setup", 5),
        ("solve", 2, "rebuilt_levels", "tfms_after_down", 1e-10, {"nu1": 1}),
    ]
    assert int(A[0][0, 0]) == 3
    assert info["iterations"] == 3 + 3 and info["fmg"] == 0.5


def test_multilevel_fmg_converges_to_als_minimum():
    """On s = 20, R = 2 (4 levels) the combination reaches g < 1e-10, in far
    fewer cycles than ALS needs sweeps, at the fit that standalone ALS from the
    same boot factors converges to."""
    d = synth.dense_case(20, 2)
    Z = d["Z"]
    assert amg.n_levels(Z.shape, d["coarsest"]) == 4
    cs = synth.dense_coarse_start((3, 3, 3), 2, d["seed"])
    A, info = amg.multilevel_fmg(Z, d["boot"], d["tfms"], d["coarsest"], cs,
                                 setup=amg.SETUP_PARAMS_NO_NT, fas=amg.FAS_PARAMS)
    assert info["levels"] == 4
    assert info["solve"][-1] < 1e-10 and cp.grad_norm(Z, A) < 1e-10
    B, h = cp.als(Z, d["boot"], max_sweeps=3000, fit_tol=None, g_tol=1e-10)
    assert h["g"][-1] < 1e-10
    assert info["iterations"] < h["sweeps"] / 5
    assert abs(cp.fit(Z, A) - cp.fit(Z, B)) < 1e-10

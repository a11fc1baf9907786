"""Host logic of the drivers' stopping rules, with the device calls replaced by
stand-ins (no GPU): the Section 6.1 solve phase on a scripted g sequence."""
import math

import pytest

from paper_1111_6091_amd import drivers


class _Factors:
    """Stand-in factor set: a value that cycles overwrite."""

    def __init__(self, v=0):
        self.v = v

    def clone(self):
        return _Factors(self.v)


def _run(monkeypatch, gs, max_cycles=20):
    """solve_phase where cycle k yields g = gs[k] (gs[0]: the start)."""
    seq = iter(gs)
    calls = {"rebuild": 0, "cycle": 0}
    monkeypatch.setattr(drivers, "grad_norm", lambda ctx, Z, A: next(seq))

    def vcycle(ctx, levels, A, **fas):
        calls["cycle"] += 1
        A.v = calls["cycle"]
    monkeypatch.setattr(drivers.api, "cp_fas_vcycle", vcycle)

    def rebuild(ctx, Z, A, tfms, coarsest, nu1=5):
        calls["rebuild"] += 1
        return "rebuilt-levels", None
    monkeypatch.setattr(drivers, "down_sweep", rebuild)
    monkeypatch.setattr(drivers, "_copy_factors", lambda dst, src: setattr(dst, "v", src.v))
    A = _Factors()
    levels, hist, rebuilt = drivers.solve_phase(None, None, A, "levels", None, None, tau=1e-10,
                                                max_cycles=max_cycles)
    return A, hist, rebuilt, calls


def test_solve_phase_stops_below_tau(monkeypatch):
    A, hist, rebuilt, calls = _run(monkeypatch, [1.0, 1e-3, 1e-6, 1e-11])
    assert hist == [1e-3, 1e-6, 1e-11] and not rebuilt and A.v == 3


def test_solve_phase_rebuilds_once_on_stagnation_after_five_cycles(monkeypatch):
    # cycles 1-5 accepted (cycle 4 rises, before the check starts); cycle 6 does
    # not lower g -> discarded and rebuilt; cycle 7 goes on from the old iterate
    gs = [1.0, 0.5, 0.4, 0.3, 0.35, 0.2, 0.25, 1e-11]
    A, hist, rebuilt, calls = _run(monkeypatch, gs)
    assert rebuilt and calls["rebuild"] == 1
    assert hist == [0.5, 0.4, 0.3, 0.35, 0.2, 1e-11]
    assert A.v == 7


def test_solve_phase_discards_a_diverged_cycle(monkeypatch):
    # a NaN g at cycle 2 is discarded (the one rebuild); a second one ends the
    # phase with the factors of the last finite cycle
    gs = [1.0, 0.5, float("nan"), 0.4, float("nan"), 0.3]
    A, hist, rebuilt, calls = _run(monkeypatch, gs)
    assert rebuilt and calls["rebuild"] == 1
    assert hist == [0.5, 0.4] and all(math.isfinite(g) for g in hist)
    assert A.v == 3   # cycle 3's factors; cycles 2 and 4 were discarded

"""Parity at the workloads' full sizes, in the launch configuration the benchmark
times (autotuned plans), against the oracle and its stored results.

Final fits are compared at the oracle's own sweep (cycle) count: near the end of
a slow ALS run the fit still moves by about the stopping tolerance per sweep, so
two runs that stop one or two sweeps apart differ by a few times that tolerance
for reasons that have nothing to do with arithmetic.  The stopping rule itself
is checked separately (the device solve must stop within a few sweeps of the
oracle).

  256^3 R=10 (collinearity 0.9): MTTKRP of every mode; FP64 ALS at the oracle's
      1929 sweeps to 1e-12; the mixed form to the FP64 final fit to 1e-10
      (tests/golden/als_c3_256cube_r10.json).
  64^4 R=8: MTTKRP of every mode; FP64 ALS at the oracle's sweep count to
      1e-12; the mixed form to the FP64 final fit to 1e-10; the first 3-level
      CP-FAS V-cycles (tests/golden/als_c4_64quart_r8.json, fas_c4_64quart_r8.json).
  128^3 R=5, 4 levels: transfer operators, coarse tensors and one CP-FAS V-cycle
      on the hierarchy of the oracle's setup phase; ALS and CP-FAS at the
      oracle's counts to 1e-12; the mixed CP-FAS solve with its FP64 finishing
      cycles to the FP64 final fit to 1e-10 (tests/golden/fas_c2_128cube_r5.json).
  20^3 R=3: ALS, down-sweep operators, one V-cycle, ALS to convergence
      (tests/golden/c1_20cube_r3_pipeline.json).
  512 tensors x 4 restarts: the whole batch for a fixed number of sweeps against
      the oracle; the whole batch in the mixed form to its stopping rules against
      the oracle's final fits of 16 sampled problems
      (tests/golden/batch_sampled_final_fits.json).
"""
import json
import os

import numpy as np
import pytest

from oracle import amg, cp
from paper_1111_6091_amd import synth
from tests.gpu_util import ROOT, ctx as make_ctx, elem_err, mttkrp_err, say, sync

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"tests/golden/{name} not generated")
    with open(path) as f:
        return json.load(f)


def _run_sweeps(C, Zd, A, count, prec, chunk=256):
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_SOLVE_CHOL
    done = 0
    while done < count:
        k = min(chunk, count - done)
        api.cp_als_sweep(C, Zd, A, None, k, CP_SOLVE_CHOL, 10, True, prec)
        done += k


def _rel(a, b):
    return abs(a - b) / abs(b)


@pytest.fixture(scope="module")
def C():
    return make_ctx()


@pytest.fixture(scope="module")
def c3(C):
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED
    Z, _, spec = synth.workload("c3_256cube_r10")
    A0 = synth.uniform_start(Z.shape, spec["R"], spec["seed"])
    Zd = api.DeviceTensor.from_numpy(C, Z, fp32=True)
    At = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    for prec in (CP_MIXED, CP_FP64):
        api.cp_autotune(C, Zd, At, prec, 5)
    sync()
    return Z, A0, spec, Zd


@pytest.mark.parametrize("mixed", [False, True])
def test_c3_mttkrp_every_mode(C, c3, mixed):
    import torch
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED
    Z, A0, spec, Zd = c3
    say(f"c3 mttkrp mixed={mixed}")
    A = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    for n in range(3):
        M = torch.empty((Z.shape[n], spec["R"]), dtype=torch.float64, device="cuda")
        api.cp_mttkrp(C, Zd, A, n, M, CP_MIXED if mixed else CP_FP64)
        sync()
        e = mttkrp_err(M.cpu().numpy(), Z, A0, n)
        say(f"  mode {n}: element-wise err {e:.2e}")
        assert e < (2e-5 if mixed else 1e-12)


def test_c3_tuned_plans_cover_the_tile_storing_launch_and_round_trip(C, c3):
    """The autotuner keeps a configuration for the mode-1 launch that stores
    the stage-1 tiles (key suffix ;y), and a second context that imports the
    exported plans runs bit-identical sweeps."""
    import torch
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_MIXED, CP_SOLVE_CHOL
    Z, A0, spec, Zd = c3
    text = api.cp_plans_export(C)
    keys = [ln.split()[0] for ln in text.strip().splitlines()]
    say(f"tuned plans: {len(keys)} keys")
    for prec in ("mixed", "fp64"):
        assert any(k.endswith(f"n=1;R=10;prec={prec};y") for k in keys), keys
    C2 = make_ctx()
    api.cp_plans_import(C2, text)
    outs = []
    for ctx in (C, C2):
        A = api.DeviceFactors.from_numpy(ctx, A0, fp32=True)
        fh = torch.zeros(3, dtype=torch.float64, device="cuda")
        api.cp_als_sweep(ctx, Zd, A, None, 3, CP_SOLVE_CHOL, 10, True, CP_MIXED, fh)
        sync()
        outs.append([a.copy() for a in A.to_numpy()] + [fh.cpu().numpy()])
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


def test_c3_als_sweeps_match_oracle(C, c3):
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_FP64, CP_SOLVE_CHOL
    Z, A0, spec, Zd = c3
    say("c3 fp64 sweeps")
    A = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    api.cp_als_sweep(C, Zd, A, None, 3, CP_SOLVE_CHOL, 10, True, CP_FP64)
    sync()
    ref = [a.copy() for a in A0]
    for _ in range(3):
        ref = cp.als_sweep(Z, ref)
    got = A.to_numpy()
    for n in range(3):
        assert elem_err(got[n], ref[n]) < 1e-9, (n, elem_err(got[n], ref[n]))


def test_c3_fp64_final_fit_matches_oracle(C, c3):
    """FP64 ALS at the oracle's sweep count lands on the oracle's fit to 1e-12;
    the device's own stopping rule ends within a few sweeps of the oracle's."""
    from paper_1111_6091_amd import api, drivers
    from paper_1111_6091_amd._lib import CP_FP64
    Z, A0, spec, Zd = c3
    g = _golden("als_c3_256cube_r10.json")
    say(f"c3 fp64: {g['sweeps']} sweeps")
    A = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    _run_sweeps(C, Zd, A, g["sweeps"], CP_FP64)
    fit = drivers.exact_fit(C, Zd, A)
    say(f"  oracle fit {g['final_fit_exact']:.16f}, device {fit:.16f}, rel {_rel(fit, g['final_fit_exact']):.2e}")
    assert _rel(fit, g["final_fit_exact"]) <= 1e-12
    A = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    r = drivers.als_solve(C, Zd, A, fit_tol=g["fit_tol"], prec=CP_FP64)
    say(f"  stopping rule: device {r.sweeps} sweeps, oracle {g['sweeps']}")
    assert r.converged and abs(r.sweeps - g["sweeps"]) <= 16
    assert C.status() == 0


def test_c3_mixed_reaches_the_fp64_fit(C, c3):
    from paper_1111_6091_amd import api, drivers
    from paper_1111_6091_amd._lib import CP_FP64
    Z, A0, spec, Zd = c3
    g = _golden("als_c3_256cube_r10.json")
    say("c3 fp64 and mixed to the 1e-12 rule")
    A = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    r64 = drivers.als_solve(C, Zd, A, fit_tol=1e-12, prec=CP_FP64)
    fit64 = drivers.exact_fit(C, Zd, A)
    A = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    rm = drivers.mixed_solve(C, Zd, A, tol32=1e-9, tol64=1e-12)
    fitm = drivers.exact_fit(C, Zd, A)
    say(f"  fp64 {r64.sweeps} sweeps fit {fit64:.16f}; mixed {rm.sweeps32}+{rm.sweeps64} fit {fitm:.16f}; "
        f"mixed vs fp64 {_rel(fitm, fit64):.2e}, vs oracle {_rel(fitm, g['final_fit_exact']):.2e}")
    assert _rel(fitm, fit64) <= 1e-10
    assert _rel(fitm, g["final_fit_exact"]) <= 1e-10
    # the FP32 phase runs past its own objective's noise floor (checked with
    # FP64-contraction fits), so most sweeps of the solve are FP32 sweeps
    assert rm.sweeps32 > rm.sweeps64
    assert C.status() == 0


@pytest.fixture(scope="module")
def c4(C):
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED
    Z, _, spec = synth.workload("c4_64quart_r8")
    A0 = synth.uniform_start(Z.shape, spec["R"], spec["seed"])
    Zd = api.DeviceTensor.from_numpy(C, Z, fp32=True)
    At = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    for prec in (CP_MIXED, CP_FP64):
        api.cp_autotune(C, Zd, At, prec, 5)
    sync()
    return Z, A0, spec, Zd


@pytest.mark.parametrize("mixed", [False, True])
def test_c4_mttkrp_every_mode(C, c4, mixed):
    import torch
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED
    Z, A0, spec, Zd = c4
    say(f"c4 mttkrp mixed={mixed}")
    A = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    for n in range(4):
        M = torch.empty((Z.shape[n], spec["R"]), dtype=torch.float64, device="cuda")
        api.cp_mttkrp(C, Zd, A, n, M, CP_MIXED if mixed else CP_FP64)
        sync()
        e = mttkrp_err(M.cpu().numpy(), Z, A0, n)
        say(f"  mode {n}: element-wise err {e:.2e}")
        assert e < (2e-5 if mixed else 1e-12)


def test_c4_als_sweeps_match_oracle(C, c4):
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_FP64, CP_SOLVE_CHOL
    Z, A0, spec, Zd = c4
    say("c4 fp64 sweeps")
    A = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    api.cp_als_sweep(C, Zd, A, None, 2, CP_SOLVE_CHOL, 10, True, CP_FP64)
    sync()
    ref = [a.copy() for a in A0]
    for _ in range(2):
        ref = cp.als_sweep(Z, ref)
    got = A.to_numpy()
    for n in range(4):
        assert elem_err(got[n], ref[n]) < 1e-9, (n, elem_err(got[n], ref[n]))


def test_c4_final_fits(C, c4):
    """FP64 ALS at the oracle's sweep count to 1e-12 of the oracle's fit; the
    mixed solve (FP32 sweeps, then FP64 refinement sweeps) to 1e-10 of the FP64
    solve's final fit."""
    from paper_1111_6091_amd import api, drivers
    from paper_1111_6091_amd._lib import CP_FP64
    Z, A0, spec, Zd = c4
    g = _golden("als_c4_64quart_r8.json")
    say(f"c4 fp64: {g['sweeps']} sweeps")
    A = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    _run_sweeps(C, Zd, A, g["sweeps"], CP_FP64)
    fit = drivers.exact_fit(C, Zd, A)
    say(f"  oracle fit {g['final_fit_exact']:.16f}, device {fit:.16f}, rel {_rel(fit, g['final_fit_exact']):.2e}")
    assert _rel(fit, g["final_fit_exact"]) <= 1e-12
    A = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    r64 = drivers.als_solve(C, Zd, A, fit_tol=1e-12, prec=CP_FP64)
    fit64 = drivers.exact_fit(C, Zd, A)
    A = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    rm = drivers.mixed_solve(C, Zd, A)
    fitm = drivers.exact_fit(C, Zd, A)
    say(f"  fp64 {r64.sweeps} sweeps fit {fit64:.16f}; mixed {rm.sweeps32}+{rm.sweeps64} fit {fitm:.16f}; "
        f"rel {_rel(fitm, fit64):.2e}")
    assert abs(r64.sweeps - g["sweeps"]) <= 16
    assert _rel(fitm, fit64) <= 1e-10
    assert C.status() == 0


@pytest.mark.parametrize("mixed", [False, True])
def test_c4_three_level_vcycles_match_oracle(C, mixed):
    """64^4 R=8, 3 levels (64 -> 32 -> 16) from the oracle's setup phase: the first
    three CP-FAS V-cycles against the oracle's (FP64 to rounding; the mixed form,
    FP32 contractions and coarse tensors, to its FP32 error), and the fit after them.
    (From this start the cycles lose fit in both implementations: the setup phase's
    operators do not represent the solution well here.)"""
    from paper_1111_6091_amd import api, drivers
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED
    g = _golden("fas_c4_64quart_r8.json")
    Z, _, spec = synth.workload("c4_64quart_r8")
    weights = [[None if w is None else np.asarray(w) for w in lv] for lv in g["weights"]]
    A = [np.asarray(a) for a in g["A_setup"]]
    prec = CP_MIXED if mixed else CP_FP64
    say(f"c4 3-level V-cycles mixed={mixed}")
    Zd = api.DeviceTensor.from_numpy(C, Z, fp32=mixed)
    dlev = drivers.build_hierarchy(C, Zd, weights, prec=prec, fp32=mixed)
    assert len(dlev) == g["levels"] == 3
    Ad = api.DeviceFactors.from_numpy(C, A, fp32=mixed)
    fits = []
    for _ in range(3):
        api.cp_fas_vcycle(C, dlev, Ad, prec=prec, **amg.FAS_PARAMS)
        fits.append(drivers.exact_fit(C, Zd, Ad))
    sync()
    say(f"  oracle fits {g['fas_fits']}; device {fits}")
    tol = 1e-6 if mixed else 1e-11
    for a, b in zip(fits, g["fas_fits"]):
        assert abs(a - b) <= tol * abs(b)
    assert C.status() == 0


@pytest.fixture(scope="module")
def c2(C):
    from paper_1111_6091_amd import api, drivers
    from paper_1111_6091_amd._lib import CP_MIXED
    g = _golden("fas_c2_128cube_r5.json")
    Z, _, spec = synth.workload("c2_128cube_r5")
    weights = [[None if w is None else np.asarray(w) for w in lv] for lv in g["weights"]]
    Zd = api.DeviceTensor.from_numpy(C, Z, fp32=True)
    dlev = drivers.build_hierarchy(C, Zd, weights, prec=CP_MIXED, fp32=True, fp64=True)
    sync()
    return g, Z, weights, Zd, dlev


def test_c2_hierarchy_and_vcycle_match_oracle(C, c2):
    from paper_1111_6091_amd import api
    g, Z, weights, Zd, dlev = c2
    levels = amg.hierarchy_from_weights(Z, weights, g["coarsest"])
    assert len(levels) == g["levels"] == 4
    A = [np.asarray(a) for a in g["A_setup"]]
    say("c2 hierarchy + one V-cycle, 4 levels")
    for l, (lv, (Zl, ph)) in enumerate(zip(levels, dlev)):
        assert elem_err(Zl.to_numpy(), lv.Z) < 1e-12, l
        for n in range(3):
            if lv.Phat[n] is not None:
                assert elem_err(ph[n].cpu().numpy(), lv.Phat[n]) < 1e-13, (l, n)
    ref = amg.fas_vcycle(levels, amg.zeros_like_factors(A), A, **amg.FAS_PARAMS)
    Ad = api.DeviceFactors.from_numpy(C, A)
    api.cp_fas_vcycle(C, dlev, Ad, **amg.FAS_PARAMS)
    sync()
    got = Ad.to_numpy()
    for n in range(3):
        assert elem_err(got[n], ref[n]) < 1e-9, (n, elem_err(got[n], ref[n]))
    assert C.status() == 0


def test_c2_als_and_fas_final_fits_match_oracle(C, c2):
    """From the setup phase's factors: ALS at the oracle's sweep count and CP-FAS
    at the oracle's cycle count, each to 1e-12 of the oracle's fit."""
    from paper_1111_6091_amd import api, drivers
    from paper_1111_6091_amd._lib import CP_FP64
    g, Z, weights, Zd, dlev = c2
    As = [np.asarray(a) for a in g["A_setup"]]
    say(f"c2 ALS {g['als_sweeps']} sweeps, CP-FAS {g['fas_cycles']} cycles")
    A = api.DeviceFactors.from_numpy(C, As)
    _run_sweeps(C, Zd, A, g["als_sweeps"], CP_FP64)
    fa = drivers.exact_fit(C, Zd, A)
    A = api.DeviceFactors.from_numpy(C, As)
    for _ in range(g["fas_cycles"]):
        api.cp_fas_vcycle(C, dlev, A, **amg.FAS_PARAMS)
    ff = drivers.exact_fit(C, Zd, A)
    say(f"  ALS {fa:.16f} (oracle {g['als_fit']:.16f}, rel {_rel(fa, g['als_fit']):.2e}); "
        f"FAS {ff:.16f} (oracle {g['fas_fit']:.16f}, rel {_rel(ff, g['fas_fit']):.2e})")
    assert _rel(fa, g["als_fit"]) <= 1e-12
    assert _rel(ff, g["fas_fit"]) <= 1e-12
    A = api.DeviceFactors.from_numpy(C, As)
    r = drivers.fas_solve(C, dlev, Zd, A, fit_tol=g["fit_tol"], **amg.FAS_PARAMS)
    say(f"  stopping rule: device {r.sweeps} cycles, oracle {g['fas_cycles']}")
    assert r.converged and abs(r.sweeps - g["fas_cycles"]) <= 2
    assert C.status() == 0


def test_c2_mixed_fas_with_fp64_finish_reaches_the_fp64_fit(C, c2):
    """Mixed CP-FAS (FP32 contractions and coarse tensors) followed by FP64
    cycles, against the FP64 CP-FAS solve from the same start, to 1e-10.  The
    fit of successive CP-FAS cycles zigzags (the oracle's own sequence goes down
    in 165 of its 472 steps), so both solves stop only once three successive
    fit changes are within 1e-12."""
    from paper_1111_6091_amd import api, drivers
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED
    g, Z, weights, Zd, dlev = c2
    As = [np.asarray(a) for a in g["A_setup"]]
    say("c2 FP64 FAS, and mixed FAS + FP64 finish, 3-change rule")
    A = api.DeviceFactors.from_numpy(C, As, fp32=True)
    r64 = drivers.fas_solve(C, dlev, Zd, A, fit_tol=g["fit_tol"], prec=CP_FP64, window=3, max_cycles=3000,
                            **amg.FAS_PARAMS)
    A = api.DeviceFactors.from_numpy(C, As, fp32=True)
    rm = drivers.fas_solve(C, dlev, Zd, A, fit_tol=g["fit_tol"], prec=CP_MIXED, window=3, max_cycles=3000,
                           **amg.FAS_PARAMS)
    say(f"  FP64 {r64.sweeps} cycles fit {r64.final_fit:.16f}; mixed {rm.sweeps32} + FP64 {rm.sweeps64} "
        f"cycles fit {rm.final_fit:.16f}; rel {_rel(rm.final_fit, r64.final_fit):.2e}; ALS limit "
        f"{g['als_fit']:.16f}")
    assert r64.converged and rm.converged and rm.sweeps32 >= 1 and rm.sweeps64 >= 1
    assert _rel(rm.final_fit, r64.final_fit) <= 1e-10
    assert C.status() == 0


def test_c1_as_configured_matches_oracle(C):
    """20^3 R=3: 10 ALS sweeps, the oracle's down-sweep operators (20 -> 10),
    one CP-FAS V-cycle, then ALS to the stopping rule: same sweep count (to one
    sweep) and final fit to 1e-12."""
    from paper_1111_6091_amd import api, drivers
    from paper_1111_6091_amd._lib import CP_FP64
    g = _golden("c1_20cube_r3_pipeline.json")
    Z, _, spec = synth.workload("c1_20cube_r3")
    A0 = synth.uniform_start(Z.shape, spec["R"], spec["seed"], g["restart"])
    weights = [[None if w is None else np.asarray(w) for w in lv] for lv in g["weights"]]
    say("c1 pipeline")
    Zd = api.DeviceTensor.from_numpy(C, Z)
    A = api.DeviceFactors.from_numpy(C, A0)
    _run_sweeps(C, Zd, A, g["first_sweeps"], CP_FP64)
    dlev = drivers.build_hierarchy(C, Zd, weights)
    assert len(dlev) == g["levels"]
    api.cp_fas_vcycle(C, dlev, A, **amg.FAS_PARAMS)
    fc = drivers.exact_fit(C, Zd, A)
    assert _rel(fc, g["fit_after_cycle"]) <= 1e-12, (fc, g["fit_after_cycle"])
    r = drivers.als_solve(C, Zd, A, fit_tol=g["fit_tol"], prec=CP_FP64, sort_at_end=False)
    fit = drivers.exact_fit(C, Zd, A)
    say(f"  after the cycle {fc:.16f}; ALS {r.sweeps} sweeps (oracle {g['als_sweeps']}) fit {fit:.16f} "
        f"(oracle {g['final_fit_exact']:.16f}, rel {_rel(fit, g['final_fit_exact']):.2e})")
    assert abs(r.sweeps - g["als_sweeps"]) <= 1
    assert _rel(fit, g["final_fit_exact"]) <= 1e-12
    assert C.status() == 0


@pytest.fixture(scope="module")
def c5_problems():
    return synth.batched_problems(512)


def _c5_device(C, probs, fp32):
    from paper_1111_6091_amd import api
    dev = []
    for p in probs:
        Zd = api.DeviceTensor.from_numpy(C, p["Z"], fp32=fp32)
        cat = [np.hstack([p["starts"][k][n] for k in range(4)]) for n in range(3)]
        dev.append((Zd, api.DeviceFactors.from_numpy(C, cat, fp32=fp32)))
    return dev


def test_c5_whole_batch_fixed_sweeps_sampled(C, c5_problems):
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_FP64
    probs = c5_problems
    P = [int(np.prod(p["dims"])) for p in probs]
    sample = sorted({int(np.argmax(P)), int(np.argmin(P)), 257})
    say(f"c5 whole batch, 12 FP64 sweeps; sampled problems {sample}")
    dev = _c5_device(C, probs, False)
    K = 12
    fits, sweeps = api.cp_als_batched(C, dev, 4, prec=CP_FP64, tol64=0.0, max_sweeps=K, chunk=5)
    sync()
    sw = sweeps.cpu().numpy()
    assert (sw[:, :, 1] == K).all() and (sw[:, :, 0] == 0).all()
    for b in sample:
        p = probs[b]
        got = dev[b][1].to_numpy()
        for k in range(4):
            A = [a.copy() for a in p["starts"][k]]
            for _ in range(K):
                A = cp.als_sweep(p["Z"], A)
            for n in range(3):
                Gk = got[n][:, k * p["R"]:(k + 1) * p["R"]]
                assert elem_err(Gk, A[n]) < 1e-9, (b, k, n, elem_err(Gk, A[n]))
    assert C.status() == 0


def test_c5_mixed_batch_final_fits_match_oracle(C, c5_problems):
    """The whole 512 x 4 batch in the mixed form (FP32 phase, then FP64 phase)
    to its stopping rules; the final fit of every restart of 16 sampled problems
    (largest, smallest, both capped restarts, the slowest) against the oracle's
    FP64 solve from the same start, to 1e-10."""
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_MIXED
    g = _golden("batch_sampled_final_fits.json")
    probs = c5_problems
    say("c5 whole batch, mixed, to the stopping rules")
    dev = _c5_device(C, probs, True)
    fits, sweeps = api.cp_als_batched(C, dev, 4, prec=CP_MIXED, tol64=g["fit_tol"], max_sweeps=g["max_sweeps"])
    sync()
    sw = sweeps.cpu().numpy()
    worst = 0.0
    for e in g["problems"]:
        b, R = e["b"], e["R"]
        p = probs[b]
        got = dev[b][1].to_numpy()
        for row in e["restarts"]:
            k = row["restart"]
            A = [got[n][:, k * R:(k + 1) * R] for n in range(3)]
            fit = cp.fit(p["Z"], A)
            err = _rel(fit, row["final_fit_exact"])
            worst = max(worst, err)
            say(f"  problem {b} restart {k}: sweeps {sw[b, k].tolist()} (oracle {row['sweeps']}), "
                f"fit {fit:.14f} oracle {row['final_fit_exact']:.14f} rel {err:.2e}")
            assert err <= 1e-10, (b, k, err)
    say(f"  worst {worst:.2e}")
    assert C.status() == 0

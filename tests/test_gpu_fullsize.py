"""Parity at the workloads' full sizes, in the launch configuration the benchmark
times (autotuned plans), against the oracle and its stored results.

  256^3 R=10 (collinearity 0.9): MTTKRP of every mode, ALS sweeps, both forms
      reaching the oracle's final fit (tests/golden/als_c3_256cube_r10.json).
  64^4 R=8: MTTKRP of every mode (two stripe modes), ALS sweeps.
  128^3 R=5, 4 levels: transfer operators, coarse tensors and one CP-FAS V-cycle
      on the hierarchy of the oracle's setup phase; FAS solve to the oracle's fit
      (tests/golden/fas_c2_128cube_r5.json).
  512 tensors x 4 restarts: the whole batch for a fixed number of sweeps, sampled
      problems against the oracle.
"""
import json
import os

import numpy as np
import pytest

from oracle import amg, cp
from paper_1111_6091_amd import synth
from tests.gpu_util import ROOT, ctx as make_ctx, rel_err, say, sync

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(ROOT, "tests", "golden")


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
        e = rel_err(M.cpu().numpy(), cp.mttkrp(Z, A0, n))
        say(f"  mode {n}: rel err {e:.2e}")
        assert e < (2e-5 if mixed else 1e-12)


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
        assert rel_err(got[n], ref[n]) < 1e-9, (n, rel_err(got[n], ref[n]))


def test_c3_both_forms_reach_the_oracle_fit(C, c3):
    from paper_1111_6091_amd import api, drivers
    from paper_1111_6091_amd._lib import CP_FP64
    Z, A0, spec, Zd = c3
    with open(os.path.join(GOLDEN, "als_c3_256cube_r10.json")) as f:
        g = json.load(f)
    say("c3 fp64 and mixed to 1e-12")
    A = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    r64 = drivers.als_solve(C, Zd, A, fit_tol=1e-12, prec=CP_FP64)
    fit64 = drivers.exact_fit(C, Zd, A)
    A = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    rm = drivers.mixed_solve(C, Zd, A, tol32=1e-9, tol64=1e-12)
    fitm = drivers.exact_fit(C, Zd, A)
    say(f"  oracle {g['sweeps']} sweeps fit {g['final_fit_exact']:.15f}; fp64 {r64.sweeps} sweeps "
        f"fit {fit64:.15f}; mixed {rm.sweeps32}+{rm.sweeps64} fit {fitm:.15f}")
    ref = g["final_fit_exact"]
    assert abs(fit64 - ref) <= 1e-10 * ref
    assert abs(fitm - ref) <= 1e-10 * ref
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
        e = rel_err(M.cpu().numpy(), cp.mttkrp(Z, A0, n))
        say(f"  mode {n}: rel err {e:.2e}")
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
        assert rel_err(got[n], ref[n]) < 1e-9, (n, rel_err(got[n], ref[n]))


def _c2_golden():
    path = os.path.join(GOLDEN, "fas_c2_128cube_r5.json")
    if not os.path.exists(path):
        pytest.skip("tests/golden/fas_c2_128cube_r5.json not generated")
    with open(path) as f:
        return json.load(f)


def test_c2_hierarchy_and_vcycle_match_oracle(C):
    from paper_1111_6091_amd import api, drivers
    g = _c2_golden()
    Z, _, spec = synth.workload("c2_128cube_r5")
    weights = [[None if w is None else np.asarray(w) for w in lv] for lv in g["weights"]]
    levels = amg.hierarchy_from_weights(Z, weights, g["coarsest"])
    assert len(levels) == g["levels"] == 4
    A = [np.asarray(a) for a in g["A_setup"]]
    say("c2 hierarchy + one V-cycle, 4 levels")
    Zd = api.DeviceTensor.from_numpy(C, Z)
    dlev = drivers.build_hierarchy(C, Zd, weights)
    sync()
    for l, (lv, (Zl, ph)) in enumerate(zip(levels, dlev)):
        assert rel_err(Zl.to_numpy(), lv.Z) < 1e-12, l
        for n in range(3):
            if lv.Phat[n] is not None:
                assert rel_err(ph[n].cpu().numpy(), lv.Phat[n]) < 1e-13, (l, n)
    ref = amg.fas_vcycle(levels, amg.zeros_like_factors(A), A, **amg.FAS_PARAMS)
    Ad = api.DeviceFactors.from_numpy(C, A)
    api.cp_fas_vcycle(C, dlev, Ad, **amg.FAS_PARAMS)
    sync()
    got = Ad.to_numpy()
    for n in range(3):
        assert rel_err(got[n], ref[n]) < 1e-9, (n, rel_err(got[n], ref[n]))
    assert C.status() == 0


def test_c2_fas_solve_reaches_the_oracle_fit(C):
    from paper_1111_6091_amd import api, drivers
    g = _c2_golden()
    Z, _, spec = synth.workload("c2_128cube_r5")
    weights = [[None if w is None else np.asarray(w) for w in lv] for lv in g["weights"]]
    Zd = api.DeviceTensor.from_numpy(C, Z)
    dlev = drivers.build_hierarchy(C, Zd, weights)
    Ad = api.DeviceFactors.from_numpy(C, [np.asarray(a) for a in g["A_setup"]])
    say("c2 FAS solve to 1e-12")
    r = drivers.fas_solve(C, dlev, Zd, Ad, fit_tol=g["fit_tol"], **amg.FAS_PARAMS)
    say(f"  oracle {g['fas_cycles']} cycles fit {g['fas_fit']:.15f}; device {r.sweeps} cycles fit "
        f"{r.final_fit:.15f}")
    assert abs(r.final_fit - g["fas_fit"]) <= 1e-10 * abs(g["fas_fit"])


def test_c5_whole_batch_fixed_sweeps_sampled(C):
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_FP64
    probs = synth.batched_problems(512)
    P = [int(np.prod(p["dims"])) for p in probs]
    sample = sorted({int(np.argmax(P)), int(np.argmin(P)), 257})
    say(f"c5 whole batch, 12 FP64 sweeps; sampled problems {sample}")
    dev = []
    for p in probs:
        Zd = api.DeviceTensor.from_numpy(C, p["Z"])
        cat = [np.hstack([p["starts"][k][n] for k in range(4)]) for n in range(3)]
        dev.append((Zd, api.DeviceFactors.from_numpy(C, cat)))
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
                assert rel_err(Gk, A[n]) < 1e-9, (b, k, n, rel_err(Gk, A[n]))
    assert C.status() == 0


def _c4_golden():
    path = os.path.join(GOLDEN, "fas_c4_64quart_r8.json")
    if not os.path.exists(path):
        pytest.skip("tests/golden/fas_c4_64quart_r8.json not generated")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("mixed", [False, True])
def test_c4_three_level_vcycles_match_oracle(C, mixed):
    """64^4 R=8, 3 levels (64 -> 32 -> 16) from the oracle's setup phase: the first
    three CP-FAS V-cycles against the oracle's (FP64 to rounding; the mixed form,
    FP32 contractions and coarse tensors, to its FP32 error), and the fit after them."""
    from paper_1111_6091_amd import api, drivers
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED
    g = _c4_golden()
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

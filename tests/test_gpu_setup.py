"""The multiplicative setup phase (Algorithm 1), its down-sweep rebuild, FMG
(Algorithm 3) and the Section 6.1 solve driver on the device, against the
oracle's implementations of the same algorithms from the same inputs.

The device relaxes the test blocks and the boot factors as column groups of one
factor set (one pass over Z per sweep), fits the LS interpolation weights of
eqs. (19)-(20) in a kernel and builds P^, the coarse tensors and the restricted
blocks with the transfer kernels; the host only recurses and applies the
stopping rules.
"""
import numpy as np
import pytest

from oracle import amg, cp
from paper_1111_6091_amd import synth
from tests.gpu_util import ctx as make_ctx, elem_err, say, sync

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    return make_ctx()


def _dev(C, A):
    from paper_1111_6091_amd import api
    return api.DeviceFactors.from_numpy(C, A)


@pytest.mark.parametrize("dims,R,nfit", [((20, 21, 9), 3, 2), ((20, 21, 9), 3, 3), ((33, 8, 12, 6), 2, 3)])
def test_interp_weights_match_oracle(C, dims, R, nfit):
    """Eqs. (19)-(20) for every mode: block weights from each block's gradient,
    normal equations per fine point, right endpoint of even extents."""
    import torch
    from paper_1111_6091_amd import api, drivers
    say(f"interp weights dims={dims} R={R} nfit={nfit}")
    Z, _ = synth.collinear_tensor(dims, R, 0.5, 0.05, 0.0, seed=sum(dims))
    blocks = [synth.uniform_start(dims, R, 31, k) for k in range(3)]
    for k in range(3):
        for _ in range(2):
            blocks[k] = cp.als_sweep(Z, blocks[k])
    Zd = api.DeviceTensor.from_numpy(C, Z)
    P = drivers._pack([_dev(C, b) for b in blocks])
    for n in range(len(dims)):
        w = torch.full((dims[n], 2), np.nan, dtype=torch.float64, device="cuda")
        api.cp_interp_weights(C, Zd, P, 3, nfit, n, w)
        sync()
        ref = amg.build_interp(Z, blocks[:2], blocks[2], n, use_bfm=(nfit == 3)) if nfit >= 2 else None
        got = w.cpu().numpy()
        assert elem_err(got, ref) < 1e-11, (n, elem_err(got, ref))
    assert C.status() == 0


def _setup_case(dims, R, seed, nt=2):
    Z, _ = synth.collinear_tensor(dims, R, 0.6, 0.01, 0.0, seed=seed)
    A0 = synth.uniform_start(dims, R, seed, 0)
    tfms0 = [synth.uniform_start(dims, R, seed, 100 + k) for k in range(nt)]
    return Z, A0, tfms0


@pytest.mark.parametrize("dims,R,coarsest,cycles", [((20, 20, 20), 3, 10, 3), ((32, 28, 24), 3, 8, 2)])
def test_setup_phase_matches_oracle(C, dims, R, coarsest, cycles):
    """Algorithm 1 cycles (Table 1 setup parameters) with the Section 6.1 rule:
    g after every cycle, the last cycle's interpolation weights on every level,
    the boot factors and the fine test blocks against the oracle."""
    from paper_1111_6091_amd import api, drivers
    say(f"setup phase dims={dims} R={R} coarsest={coarsest} cycles={cycles}")
    Z, A0, tfms0 = _setup_case(dims, R, 41)
    crs = [coarsest] * len(dims)
    A, tfms, levels, ghist = amg.setup_phase(Z, A0, tfms0, crs, max_cycles=cycles, check_after=cycles,
                                             **amg.SETUP_PARAMS_NO_NT)
    Zd = api.DeviceTensor.from_numpy(C, Z)
    Ad = _dev(C, A0)
    Td = [_dev(C, t) for t in tfms0]
    dlev, dw, dg = drivers.setup_phase(C, Zd, Ad, Td, crs, max_cycles=cycles, check_after=cycles)
    sync()
    say(f"  oracle g {ghist}; device g {dg}")
    assert len(dg) == len(ghist) and len(dlev) == len(levels)
    for a, b in zip(dg, ghist):
        assert abs(a - b) <= 1e-8 * b
    for l, lv in enumerate(levels[:-1]):
        for n in range(len(dims)):
            if lv.weights[n] is None:
                assert dw[l][n] is None
                continue
            e = elem_err(dw[l][n].cpu().numpy(), lv.weights[n])
            assert e < 1e-7, (l, n, e)
    got = Ad.to_numpy()
    for n in range(len(dims)):
        assert elem_err(got[n], A[n], floor=1.0) < 1e-7, (n, elem_err(got[n], A[n], floor=1.0))
    for Tg, To in zip(Td, tfms):
        for n in range(len(dims)):
            assert elem_err(Tg.to_numpy()[n], To[n], floor=1.0) < 1e-7
    assert C.status() == 0


def test_down_sweep_matches_oracle(C):
    """The rebuild of Section 6.1: TFMs relaxed, boot factors only restricted,
    the weights of every level; the boot factors on the device are untouched."""
    from paper_1111_6091_amd import api, drivers
    dims, R = (24, 20, 18), 3
    say("down-sweep")
    Z, A0, tfms0 = _setup_case(dims, R, 43)
    Ab = [a.copy() for a in A0]
    for _ in range(4):
        Ab = cp.als_sweep(Z, Ab)
    crs = [6, 6, 6]
    levels, tfms = amg.down_sweep(Z, Ab, tfms0, crs)
    Zd = api.DeviceTensor.from_numpy(C, Z)
    Ad = _dev(C, Ab)
    Td = [_dev(C, t) for t in tfms0]
    dlev, dw = drivers.down_sweep(C, Zd, Ad, Td, crs)
    sync()
    assert len(dlev) == len(levels)
    for l, lv in enumerate(levels[:-1]):
        for n in range(3):
            if lv.weights[n] is not None:
                assert elem_err(dw[l][n].cpu().numpy(), lv.weights[n]) < 1e-8, (l, n)
        if l > 0:
            # built with P^ from weights that agree to about 1e-10
            assert elem_err(dlev[l][0].to_numpy(), lv.Z) < 1e-9, l
    for n in range(3):
        np.testing.assert_array_equal(Ad.to_numpy()[n], Ab[n])
        assert elem_err(Td[0].to_numpy()[n], tfms[0][n], floor=1.0) < 1e-9
    assert C.status() == 0


def test_fmg_cycle_matches_oracle(C):
    """Algorithm 3 on a 3-level hierarchy: coarsest ALS from a seeded start, then
    interpolation and one CP-FAS V-cycle per finer level."""
    from paper_1111_6091_amd import api, drivers
    dims, R = (32, 32, 32), 3
    say("fmg cycle")
    Z, _ = synth.collinear_tensor(dims, R, 0.5, 0.01, 0.0, seed=45)
    weights, cur = [], list(dims)
    for _ in range(2):
        weights.append([synth.linear_interp_weights(d) for d in cur])
        cur = [(d + 1) // 2 for d in cur]
    levels = amg.hierarchy_from_weights(Z, weights, [8, 8, 8])
    Ac0 = synth.uniform_start(levels[-1].dims, R, 45)
    ref = amg.fmg_cycle(levels, Ac0, nu=30, nu1=1, nu2=1, nuc=20, gs_iters=10)
    Zd = api.DeviceTensor.from_numpy(C, Z)
    dlev = drivers.build_hierarchy(C, Zd, weights)
    got = drivers.fmg_cycle(C, dlev, _dev(C, Ac0), nu=30, nu1=1, nu2=1, nuc=20, gs_iters=10)
    sync()
    g = got.to_numpy()
    for n in range(3):
        assert elem_err(g[n], ref[n], floor=1.0) < 1e-8, (n, elem_err(g[n], ref[n], floor=1.0))
    # the factors agree to about 1e-9 of their largest entries after 30 coarsest
    # sweeps and two V-cycles; the fit follows to the same order
    assert abs(cp.fit(Z, g) - cp.fit(Z, ref)) <= 1e-9
    assert C.status() == 0


def test_solve_phase_matches_oracle(C):
    """Section 6.1 solve cycles from a setup phase: the g history of the CP-FAS
    cycles to g < tau against the oracle's driver on the oracle's hierarchy."""
    from paper_1111_6091_amd import api, drivers
    dims, R = (20, 20, 20), 3
    say("solve phase")
    Z, A0, tfms0 = _setup_case(dims, R, 47)
    crs = [10, 10, 10]
    A, tfms, levels, _ = amg.setup_phase(Z, A0, tfms0, crs, max_cycles=2, check_after=2,
                                         **amg.SETUP_PARAMS_NO_NT)
    Af, _, ghist = amg.solve_phase(Z, A, levels, tfms, crs, tau=1e-8, max_cycles=40, **amg.FAS_PARAMS)
    Zd = api.DeviceTensor.from_numpy(C, Z)
    weights = [lv.weights for lv in levels[:-1]]
    dlev = drivers.build_hierarchy(C, Zd, [[None if w is None else np.asarray(w) for w in wl] for wl in weights])
    Ad = _dev(C, A)
    Td = [_dev(C, t) for t in tfms]
    _, dh, rebuilt = drivers.solve_phase(C, Zd, Ad, dlev, Td, crs, tau=1e-8, max_cycles=40, **amg.FAS_PARAMS)
    sync()
    say(f"  oracle {len(ghist)} cycles g {ghist[-1]:.3e}; device {len(dh)} cycles g {dh[-1]:.3e} rebuilt={rebuilt}")
    assert len(dh) == len(ghist)
    # g is a norm of a gradient that goes to zero: its absolute rounding level
    # is about 1e-14 here (u times the size of the terms it cancels)
    for a, b in zip(dh, ghist):
        assert abs(a - b) <= 1e-6 * b + 1e-13
    assert abs(cp.fit(Z, Ad.to_numpy()) - cp.fit(Z, Af)) <= 1e-10
    assert C.status() == 0

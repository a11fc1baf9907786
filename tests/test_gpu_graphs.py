"""CP-FAS V-cycles replayed from a recorded HIP graph against the same cycles
launched kernel by kernel (the graph holds the very same launches, so every
replay must agree bit for bit).  Between the replays the program does eager work
of its own (objective evaluations, a plain MTTKRP) and synchronizes."""
import numpy as np
import pytest
import torch

from oracle import amg, cp
from paper_1111_6091_amd import synth
from tests.gpu_util import ctx as make_ctx, say, sync

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,R,nlev,mixed", [((32, 32, 32), 3, 3, False), ((40, 36, 24), 4, 3, True),
                                               ((20, 20, 20), 3, 2, False)])
def test_vcycle_graph_replays_match_eager_cycles(dims, R, nlev, mixed):
    from paper_1111_6091_amd import api, drivers
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED, CP_OPT_GRAPHS
    say(f"graph replays dims={dims} R={R} levels={nlev} mixed={mixed}")
    prec = CP_MIXED if mixed else CP_FP64
    Z, _ = synth.collinear_tensor(dims, R, 0.6, 0.01, 0.0, seed=21)
    A0, _ = cp.als(Z, synth.uniform_start(dims, R, 21), max_sweeps=5, fit_tol=0.0, sort_at_end=False)
    weights, cur = [], list(dims)
    for _ in range(nlev - 1):
        weights.append([synth.linear_interp_weights(d) for d in cur])
        cur = [(d + 1) // 2 for d in cur]
    C = make_ctx()
    Zd = api.DeviceTensor.from_numpy(C, Z, fp32=True)
    dlev = drivers.build_hierarchy(C, Zd, weights, prec=prec, fp32=True, fp64=True)
    K = 4
    # eager: graphs off
    C.set_option(CP_OPT_GRAPHS, 0)
    Ae = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    eager = []
    for _ in range(K):
        api.cp_fas_vcycle(C, dlev, Ae, prec=prec, nuc=20)
        sync()
        eager.append(Ae.to_numpy())
    # recorded once, replayed K - 1 times, with eager work in between
    C.set_option(CP_OPT_GRAPHS, 1)
    Ag = api.DeviceFactors.from_numpy(C, A0, fp32=True)
    f = torch.zeros(1, dtype=torch.float64, device="cuda")
    M = torch.zeros((dims[0], R), dtype=torch.float64, device="cuda")
    for k in range(K):
        api.cp_fas_vcycle(C, dlev, Ag, prec=prec, nuc=20)
        api.cp_objective(C, Zd, Ag, exact=True, f=f)
        api.cp_mttkrp(C, Zd, Ag, 0, M, CP_FP64)
        sync()
        got = Ag.to_numpy()
        for n in range(3):
            assert np.array_equal(got[n], eager[k][n]), (k, n, np.max(np.abs(got[n] - eager[k][n])))
        assert f.item() == pytest.approx(cp.objective(Z, got), rel=1e-11)
    assert C.status() == 0

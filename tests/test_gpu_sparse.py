"""Sparse finest level (Section 6.2) on the device: the MTTKRP over stored
entries, ALS sweeps, g and f, the restriction that makes the first coarse
tensor dense, the CP-FAS V-cycle with a sparse level 0 and the Section 6.1
'Multilevel' driver, all against the oracle (dense definitions on the
densified tensor, or the oracle's coordinate-form MTTKRP at full Table 2
sizes).  Also dense restrictions whose GEMM launches need more than 65535
batch entries or column tiles."""
import numpy as np
import pytest
import torch

from oracle import amg, cp
from paper_1111_6091_amd import synth
from tests.gpu_util import ctx as make_ctx, elem_err, say, scaled_err, sync

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def C():
    return make_ctx()


def _sp(C, idx, vals, dims):
    from paper_1111_6091_amd import api
    return api.SparseTensor.from_coo(C, idx, vals, dims)


def _dev(C, A):
    from paper_1111_6091_amd import api
    return api.DeviceFactors.from_numpy(C, A)


def _mttkrp_check(C, idx, vals, dims, R, seed, tol=1e-12):
    from paper_1111_6091_amd import api
    rng = np.random.default_rng(seed)
    A = [rng.standard_normal((d, R)) for d in dims]
    Zs = _sp(C, idx, vals, dims)
    Ad = _dev(C, A)
    absA = [np.abs(a) for a in A]
    for n in range(len(dims)):
        M = torch.full((dims[n], R), np.nan, dtype=torch.float64, device="cuda")
        api.cp_mttkrp(C, Zs, Ad, n, M)
        M2 = torch.full((dims[n], R), np.nan, dtype=torch.float64, device="cuda")
        api.cp_mttkrp(C, Zs, Ad, n, M2)
        sync()
        ref = cp.mttkrp_coo(idx, vals, dims, A, n)
        scale = cp.mttkrp_coo(idx, np.abs(vals), dims, absA, n)
        # an output is a sum of (entries in its row) terms: FP64 sums of up to
        # ~10^4 terms stay within about 1e-12 of the sum of their magnitudes
        assert scaled_err(M.cpu().numpy(), ref, scale) < tol, n
        assert torch.equal(M, M2)   # fixed reduction order: bit-identical repeats


@pytest.mark.parametrize("N,s,R", [(4, 20, 6), (4, 50, 4), (6, 20, 4), (8, 10, 3), (8, 10, 17)])
def test_sparse_mttkrp_laplacian_full_size(C, N, s, R):
    """Table 2's tensors at their full sizes (nnz up to 82000), every mode."""
    say(f"sparse mttkrp laplacian N={N} s={s} R={R}")
    idx, vals, dims = synth.laplacian_coo(N // 2, s)
    _mttkrp_check(C, idx, vals, dims, R, seed=N * s + R)
    assert C.status() == 0


@pytest.mark.parametrize("R", [5, 32])
def test_sparse_mttkrp_ragged_rows(C, R):
    """Uneven rows: one long row split over many workgroups, empty rows, an
    extent-1 mode, entries given in no particular order."""
    say(f"sparse mttkrp ragged R={R}")
    rng = np.random.default_rng(R)
    dims = (37, 1, 300)
    # row 3 of mode 0 holds every (3, 0, k); scattered entries elsewhere
    a = np.stack([np.full(300, 3), np.zeros(300, int), np.arange(300)], axis=1)
    P = 37 * 300
    lin = rng.choice(P, size=2000, replace=False)
    b = np.stack([lin % 37, np.zeros(2000, int), lin // 37], axis=1)
    b = b[(b[:, 0] != 3) & (b[:, 0] % 5 != 1)]          # rows 1, 6, 11, ... stay empty
    idx = np.concatenate([a, b]).astype(np.int32)
    idx = idx[rng.permutation(idx.shape[0])]
    vals = rng.standard_normal(idx.shape[0])
    _mttkrp_check(C, idx, vals, dims, R, seed=R + 1)
    # a single very long row: 40000 entries in one mode-0 index
    dims2 = (2, 200, 200)
    lin2 = rng.choice(200 * 200, size=40000, replace=False)
    idx2 = np.stack([np.zeros(40000, int), lin2 % 200, lin2 // 200], axis=1).astype(np.int32)
    _mttkrp_check(C, idx2, rng.standard_normal(40000), dims2, R, seed=R + 2)
    assert C.status() == 0


def test_sparse_als_sweeps_and_objective_match_oracle(C):
    """ALS sweeps on the N = 4, s = 10 Laplacian (sparse form) against the
    oracle on the dense array; then g (eq. (30)) and the fused f."""
    from paper_1111_6091_amd import api
    say("sparse als sweeps + objective")
    c = synth.laplacian_case(4, 10, 3)
    Z = synth.coo_to_dense(c["idx"], c["vals"], c["shape"])
    Zs = _sp(C, c["idx"], c["vals"], c["shape"])
    assert Zs.norm2.item() == pytest.approx(float(np.sum(Z * Z)), rel=1e-15)
    Ad = _dev(C, c["boot"])
    K = 8
    fh = torch.zeros(K, dtype=torch.float64, device="cuda")
    api.cp_als_sweep(C, Zs, Ad, None, K, api.CP_SOLVE_CHOL, 10, True, api.CP_FP64, fh)
    sync()
    A, fref = c["boot"], []
    for _ in range(K):
        A = cp.als_sweep(Z, A)
        fref.append(cp.objective(Z, A))
    got = Ad.to_numpy()
    for n in range(4):
        assert elem_err(got[n], A[n]) < 1e-9, (n, elem_err(got[n], A[n]))
    np.testing.assert_allclose(fh.cpu().numpy(), fref, rtol=1e-10)
    f = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.zeros(1, dtype=torch.float64, device="cuda")
    api.cp_objective(C, Zs, Ad, exact=True, f=f, g=g)
    sync()
    assert g.item() == pytest.approx(cp.grad_norm(Z, got), rel=1e-10)
    assert f.item() == pytest.approx(cp.objective(Z, got), rel=1e-11)
    assert C.status() == 0


@pytest.mark.parametrize("N,s,mask", [(4, 10, (1, 1, 1, 1)), (6, 6, (1, 0, 1, 0, 1, 1)), (8, 4, (1,) * 8),
                                      (4, 9, (0, 0, 0, 0))])
def test_sparse_restrict_matches_oracle(C, N, s, mask):
    """Coarse tensor eq. (15) from the sparse form against the oracle's mode
    products on the dense array (no coarsened mode: the dense copy itself)."""
    from paper_1111_6091_amd import api
    say(f"sparse restrict N={N} s={s} mask={mask}")
    idx, vals, dims = synth.laplacian_coo(N // 2, s)
    Z = synth.coo_to_dense(idx, vals, dims)
    phs = [amg.transfer(amg.interp_from_weights(d, synth.linear_interp_weights(d)))[2] if m else None
           for d, m in zip(dims, mask)]
    phd = [None if p is None else torch.from_numpy(p).cuda() for p in phs]
    ref = amg.restrict_tensor(Z, [None if p is None else p.T for p in phs])
    Zs = _sp(C, idx, vals, dims)
    Zc = api.DeviceTensor.empty(ref.shape)
    Zf = api.DeviceTensor.empty(ref.shape)
    api.cp_restrict(C, Zs, phd, Zc, api.CP_FP64)
    wd = [torch.from_numpy(synth.linear_interp_weights(d)).cuda() if m else None for d, m in zip(dims, mask)]
    api.cp_restrict_factored(C, Zs, wd, Zf, api.CP_FP64)
    sync()
    if not any(mask):
        np.testing.assert_array_equal(Zc.to_numpy(), Z)
        np.testing.assert_array_equal(Zf.to_numpy(), Z)
        return
    scale = amg.restrict_tensor(np.abs(Z), [None if p is None else np.abs(p.T) for p in phs])
    assert scaled_err(Zc.to_numpy(), ref, scale) < 1e-13
    assert scaled_err(Zf.to_numpy(), ref, scale) < 1e-13


@pytest.mark.parametrize("dims,mask", [((40, 4, 70000), (1, 1, 0)), ((3, 4400000), (1, 0)),
                                       ((5, 12, 12, 12, 12, 12), (1, 1, 1, 1, 1, 1))])
def test_dense_restrict_large_grids(C, dims, mask):
    """Mode products whose launches exceed 65535 batch entries (40 x 4 x 70000,
    mode 1), 65535 column tiles (3 x 4.4M, mode 0), and short leading extents
    (order 6) against the oracle."""
    from paper_1111_6091_amd import api
    say(f"dense restrict dims={dims} mask={mask}")
    rng = np.random.default_rng(len(dims))
    Z = rng.standard_normal(dims)
    phs = [amg.transfer(amg.interp_from_weights(d, synth.linear_interp_weights(d)))[2] if m else None
           for d, m in zip(dims, mask)]
    phd = [None if p is None else torch.from_numpy(p).cuda() for p in phs]
    ref = amg.restrict_tensor(Z, [None if p is None else p.T for p in phs])
    Zd = api.DeviceTensor.from_numpy(C, Z)
    Zc = api.DeviceTensor.empty(ref.shape)
    api.cp_restrict(C, Zd, phd, Zc, api.CP_FP64)
    sync()
    scale = amg.restrict_tensor(np.abs(Z), [None if p is None else np.abs(p.T) for p in phs])
    assert scaled_err(Zc.to_numpy(), ref, scale) < 1e-13


@pytest.mark.parametrize("N,s,R,crs", [(4, 12, 3, 6), (6, 6, 2, 3)])
def test_fas_vcycle_sparse_level0(C, N, s, R, crs):
    """One CP-FAS V-cycle whose finest level is the sparse Laplacian: against
    the oracle's V-cycle on the dense array, and against the device's own
    V-cycle with a dense level 0."""
    from paper_1111_6091_amd import api, drivers
    say(f"fas vcycle sparse level 0 N={N} s={s} R={R}")
    c = synth.laplacian_case(N, s, R)
    Z = synth.coo_to_dense(c["idx"], c["vals"], c["shape"])
    # a start 20 ALS sweeps in: from 3 sweeps the cycle on these fixed linear
    # transfers diverges (factor entries near 1e14 after one cycle)
    A0 = c["boot"]
    for _ in range(20):
        A0 = cp.als_sweep(Z, A0)
    weights = [[synth.linear_interp_weights(s)] * N]
    levels = amg.hierarchy_from_weights(Z, weights, [crs] * N)
    assert len(levels) == 2
    ref = amg.fas_vcycle(levels, amg.zeros_like_factors(A0), A0, nu1=1, nu2=1, nuc=20)
    Zs = _sp(C, c["idx"], c["vals"], c["shape"])
    Zd = api.DeviceTensor.from_numpy(C, Z)
    outs = []
    for top in (Zs, Zd):
        dlev = drivers.build_hierarchy(C, top, weights)
        Ad = _dev(C, A0)
        api.cp_fas_vcycle(C, dlev, Ad, nu1=1, nu2=1, nuc=20)
        sync()
        outs.append(Ad.to_numpy())
    for got in outs:
        for n in range(N):
            assert elem_err(got[n], ref[n]) < 1e-9, (n, elem_err(got[n], ref[n]))
    # the two device paths sum each MTTKRP in different orders (per stored
    # entry; dense modes >= 2 through the dimension tree's stage-1 tiles), and
    # the cycle's 20 coarse sweeps amplify last-bit differences on this
    # Laplacian start: they agree to 1e-10 (and each with the oracle to 1e-9)
    for n in range(N):
        assert elem_err(outs[0][n], outs[1][n]) < 1e-10, (n, elem_err(outs[0][n], outs[1][n]))
    assert C.status() == 0


@pytest.mark.parametrize("N,s,R,crs", [(4, 20, 4, None), (6, 8, 2, 5), (8, 5, 2, 3)])
def test_multilevel_laplacian_matches_oracle(C, N, s, R, crs):
    """Section 6.1 'Multilevel' (setup cycles, then CP-FAS solve cycles to
    g < 1e-10) with the sparse finest level: Table 2's test 1 (N = 4, s = 20,
    R = 4, 2 levels) and order-6 and order-8 Laplacians whose coarse levels are
    dense order-6 and order-8 tensors; the g after every cycle, the cycle
    counts and the final fit against the oracle's driver on the dense array."""
    from paper_1111_6091_amd import drivers
    say(f"multilevel laplacian N={N} s={s} R={R}")
    c = synth.laplacian_case(N, s, R)
    crs = c["coarsest"] if crs is None else [crs] * N
    Z = synth.coo_to_dense(c["idx"], c["vals"], c["shape"])
    A, ref = amg.multilevel(Z, c["boot"], c["tfms"], crs, setup=amg.SETUP_PARAMS_NO_NT, fas=amg.FAS_PARAMS)
    Zs = _sp(C, c["idx"], c["vals"], c["shape"])
    Ad = _dev(C, c["boot"])
    Td = [_dev(C, t) for t in c["tfms"]]
    got = drivers.multilevel(C, Zs, Ad, Td, crs, fas=amg.FAS_PARAMS)
    sync()
    say(f"  oracle it={ref['iterations']} ({len(ref['setup'])}+{len(ref['solve'])}) "
        f"device it={got['iterations']} ({len(got['setup'])}+{len(got['solve'])})")
    assert got["levels"] == ref["levels"] == 2
    assert len(got["setup"]) == len(ref["setup"])
    for a, b in zip(got["setup"], ref["setup"]):
        assert abs(a - b) <= 1e-8 * b + 1e-13
    assert got["rebuilt"] == ref["rebuilt"]
    assert len(got["solve"]) == len(ref["solve"])
    for a, b in zip(got["solve"], ref["solve"]):
        assert abs(a - b) <= 1e-6 * b + 1e-13
    assert abs(cp.fit(Z, Ad.to_numpy()) - cp.fit(Z, A)) <= 1e-10
    assert C.status() == 0

"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded inputs.

Tolerances: FP64 paths differ from the oracle only by summation order, so
results agree to ~1e-13 relative; tests use 1e-11 for single calls and 1e-12 on
fits.  Mixed-precision contractions (FP32 GEMM, FP32 accumulation over at most
the contracted mode length) are compared at 2e-5 relative.
"""
import numpy as np
import pytest

from oracle import amg, cp
from paper_1111_6091_amd import synth
from tests.gpu_util import ctx as make_ctx, elem_err, mttkrp_err, say, scaled_err, sync

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def C():
    from paper_1111_6091_amd import api  # noqa: F401  (fails loudly if the library is missing)
    return make_ctx()


def dev_inputs(C, Z, A, fp32=False):
    from paper_1111_6091_amd import api
    return api.DeviceTensor.from_numpy(C, Z, fp32=fp32), api.DeviceFactors.from_numpy(C, A, fp32=fp32)


MTTKRP_SHAPES = [
    ((20, 20, 20), 3), ((5, 7, 9), 2), ((64, 33, 17), 5), ((3, 4, 5, 6), 4), ((12, 10, 9, 11), 8),
    ((37, 19, 23), 16), ((16, 16, 16), 20), ((128, 64, 8), 10), ((7, 130, 5), 3), ((9, 8), 3),
]


@pytest.mark.parametrize("dims,R", MTTKRP_SHAPES)
def test_mttkrp_fp64_matches_oracle(C, dims, R):
    from paper_1111_6091_amd import api
    say(f"mttkrp fp64 dims={dims} R={R}")
    rng = np.random.default_rng(sum(dims) + R)
    Z = rng.standard_normal(dims)
    A = [rng.standard_normal((d, R)) for d in dims]
    Zd, Ad = dev_inputs(C, Z, A)
    for n in range(len(dims)):
        M = torch.zeros((dims[n], R), dtype=torch.float64, device="cuda")
        api.cp_mttkrp(C, Zd, Ad, n, M)
        sync()
        e = mttkrp_err(M.cpu().numpy(), Z, A, n)
        assert e < 1e-12, (n, e)


# the last two shapes contract modes longer than 256 (mode 1 for n = 0, mode 0
# for n >= 1): the FP32 accumulation runs over pieces of at most 256 entries
# that are added in FP64, which is what keeps the error within K u32 for K <= 256
@pytest.mark.parametrize("dims,R", [((20, 20, 20), 3), ((64, 33, 17), 5), ((12, 10, 9, 11), 8),
                                    ((37, 19, 23), 16), ((16, 16, 16), 20), ((900, 700, 3), 5),
                                    ((600, 300, 4, 3), 4)])
def test_mttkrp_mixed_matches_oracle(C, dims, R):
    from paper_1111_6091_amd import api
    say(f"mttkrp mixed dims={dims} R={R}")
    rng = np.random.default_rng(7 + R)
    Z = rng.standard_normal(dims)
    A = [rng.standard_normal((d, R)) for d in dims]
    Zd, Ad = dev_inputs(C, Z, A, fp32=True)
    for n in range(len(dims)):
        M = torch.zeros((dims[n], R), dtype=torch.float64, device="cuda")
        api.cp_mttkrp(C, Zd, Ad, n, M, prec=api.CP_MIXED)
        sync()
        e = mttkrp_err(M.cpu().numpy(), Z, A, n)
        assert e < 2e-5, (n, e)


def test_mttkrp_deterministic(C):
    from paper_1111_6091_amd import api
    rng = np.random.default_rng(3)
    dims, R = (64, 48, 40), 7
    Z = rng.standard_normal(dims)
    A = [rng.standard_normal((d, R)) for d in dims]
    Zd, Ad = dev_inputs(C, Z, A)
    for n in range(3):
        M1 = torch.zeros((dims[n], R), dtype=torch.float64, device="cuda")
        M2 = torch.zeros_like(M1)
        api.cp_mttkrp(C, Zd, Ad, n, M1)
        api.cp_mttkrp(C, Zd, Ad, n, M2)
        sync()
        assert torch.equal(M1, M2)


def test_norm2_and_objectives(C):
    from paper_1111_6091_amd import api
    say("objectives")
    Z, _ = synth.collinear_tensor((20, 21, 22), 3, 0.5, 0.05, 0.0, seed=4)
    A = synth.uniform_start(Z.shape, 3, 4)
    Zd, Ad = dev_inputs(C, Z, A)
    sync()
    assert Zd.norm2.item() == pytest.approx(float(np.sum(Z * Z)), rel=1e-13)
    f = torch.zeros(1, dtype=torch.float64, device="cuda")
    ff = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = torch.zeros(1, dtype=torch.float64, device="cuda")
    api.cp_objective(C, Zd, Ad, exact=True, f=f, g=g)
    api.cp_objective(C, Zd, Ad, exact=False, f=ff)
    sync()
    assert f.item() == pytest.approx(cp.objective(Z, A), rel=1e-12)
    assert ff.item() == pytest.approx(cp.objective(Z, A), rel=1e-10)
    assert g.item() == pytest.approx(cp.grad_norm(Z, A), rel=1e-11)


@pytest.mark.parametrize("dims,R", [((600, 8, 3), 8), ((2, 400, 400), 32), ((5, 6, 7, 8), 4)])
def test_exact_objective_matches_oracle(C, dims, R):
    """f = 1/2 ||Z - [[A]]||^2 (eq. (2)) by the residual pass, against the oracle:
    A^(0) too large for the kernel's LDS copy (600 x 8), fibres whose weights
    need several LDS groups per block (rank 32 over 160000 fibres), order 4."""
    from paper_1111_6091_amd import api
    say(f"exact objective dims={dims} R={R}")
    rng = np.random.default_rng(sum(dims) + R)
    Z = rng.standard_normal(dims)
    A = [rng.standard_normal((d, R)) / np.sqrt(R) for d in dims]
    Zd, Ad = dev_inputs(C, Z, A)
    f = torch.zeros(1, dtype=torch.float64, device="cuda")
    api.cp_objective(C, Zd, Ad, exact=True, f=f)
    sync()
    assert f.item() == pytest.approx(cp.objective(Z, A), rel=1e-12)
    assert C.status() == 0


@pytest.mark.parametrize("dims,R,seed", [((20, 20, 20), 3, 1), ((17, 9, 13), 4, 2), ((8, 9, 10, 7), 3, 3)])
def test_als_sweeps_track_oracle(C, dims, R, seed):
    from paper_1111_6091_amd import api
    say(f"als trajectory dims={dims} R={R}")
    Z, _ = synth.collinear_tensor(dims, R, 0.5, 0.01, 0.0, seed=seed)
    A0 = synth.uniform_start(dims, R, seed)
    Zd, Ad = dev_inputs(C, Z, A0)
    K = 12
    fh = torch.zeros(K, dtype=torch.float64, device="cuda")
    api.cp_als_sweep(C, Zd, Ad, None, K, api.CP_SOLVE_CHOL, 10, True, api.CP_FP64, fh)
    sync()
    A = A0
    fref = []
    for _ in range(K):
        A = cp.als_sweep(Z, A)
        fref.append(cp.objective(Z, A))
    got = Ad.to_numpy()
    for n in range(len(dims)):
        assert elem_err(got[n], A[n]) < 1e-9, (n, elem_err(got[n], A[n]))
    np.testing.assert_allclose(fh.cpu().numpy(), fref, rtol=1e-9)
    assert C.status() == 0


@pytest.mark.parametrize("dims,R", [((8, 5, 80, 256), 2), ((160, 24, 40), 20), ((16, 3, 5, 6, 7), 1)])
def test_dimension_tree_sweeps_track_oracle(C, dims, R):
    """FP64 sweeps with and without the dimension tree against the oracle.  The
    shapes reach the Y-contracting launches' edge cases: rest-index chunks of
    32 plus a ragged one per workgroup (order 4, last split shorter), Y rows
    fewer than one round of the workgroup (I1 = 5, 3), 17..32 columns, one
    column, and weights from two other stripe modes (order 5)."""
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_OPT_DIMTREE
    say(f"dimension-tree sweeps dims={dims} R={R}")
    Z, _ = synth.collinear_tensor(dims, R, 0.5, 0.01, 0.0, seed=7)
    A0 = synth.uniform_start(dims, R, 7)
    K = 3
    A = A0
    fref = []
    for _ in range(K):
        A = cp.als_sweep(Z, A)
        fref.append(cp.objective(Z, A))
    try:
        for tree in (1, 0):
            C.set_option(CP_OPT_DIMTREE, tree)
            Zd, Ad = dev_inputs(C, Z, A0)
            fh = torch.zeros(K, dtype=torch.float64, device="cuda")
            api.cp_als_sweep(C, Zd, Ad, None, K, api.CP_SOLVE_CHOL, 10, True, api.CP_FP64, fh)
            sync()
            got = Ad.to_numpy()
            for n in range(len(dims)):
                assert elem_err(got[n], A[n]) < 1e-9, (tree, n, elem_err(got[n], A[n]))
            np.testing.assert_allclose(fh.cpu().numpy(), fref, rtol=1e-9)
    finally:
        C.set_option(CP_OPT_DIMTREE, 1)
    assert C.status() == 0


@pytest.mark.parametrize("dims,R", [((160, 24, 40), 20), ((16, 3, 5, 6, 7), 1)])
def test_dimension_tree_mixed_matches_per_mode_passes(C, dims, R):
    """Mixed-form sweeps with the dimension tree (stage-1 tiles kept in FP32)
    against the mixed form with one pass over Z per mode, and against the
    oracle.  Each MTTKRP carries an FP32 contraction error of at most
    K u32 (K = 256 products per FP32 piece, u32 = 2^-24) relative; a solve with
    Gamma amplifies it by at most cond(Gamma), so three sweeps are allowed
    3 cond_max K u32 element-wise, cond_max taken over the oracle's Gammas."""
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_OPT_DIMTREE
    say(f"dimension-tree mixed sweeps dims={dims} R={R}")
    Z, _ = synth.collinear_tensor(dims, R, 0.5, 0.01, 0.0, seed=8)
    A0 = synth.uniform_start(dims, R, 8)
    K = 3
    A = A0
    kappa = 1.0
    for _ in range(K):
        for n in range(len(dims)):
            G = np.ones((R, R))
            for m in range(len(dims)):
                if m != n:
                    G *= A[m].T @ A[m]
            kappa = max(kappa, np.linalg.cond(G))
        A = cp.als_sweep(Z, A)
    tol = 3 * kappa * 256 * 2.0 ** -24
    outs = []
    try:
        for tree in (1, 0):
            C.set_option(CP_OPT_DIMTREE, tree)
            Zd, Ad = dev_inputs(C, Z, A0, fp32=True)
            api.cp_als_sweep(C, Zd, Ad, None, K, api.CP_SOLVE_CHOL, 10, True, api.CP_MIXED)
            sync()
            outs.append(Ad.to_numpy())
    finally:
        C.set_option(CP_OPT_DIMTREE, 1)
    for n in range(len(dims)):
        e_tree = elem_err(outs[0][n], outs[1][n])
        e_orc = elem_err(outs[0][n], A[n])
        say(f"  mode {n}: tree vs per-mode {e_tree:.1e}, vs oracle {e_orc:.1e} (bound {tol:.1e})")
        assert e_tree < tol, (n, e_tree, tol)
        assert e_orc < tol, (n, e_orc, tol)
    assert C.status() == 0


def test_als_gs_with_rhs_matches_oracle_bngs(C):
    from paper_1111_6091_amd import api
    say("bngs gs10 with F")
    dims, R = (14, 15, 16), 3
    Z, _ = synth.collinear_tensor(dims, R, 0.7, 0.02, 0.0, seed=5)
    A0 = synth.uniform_start(dims, R, 5)
    rng = np.random.default_rng(5)
    F = [0.2 * rng.standard_normal((d, R)) for d in dims]
    Zd, Ad = dev_inputs(C, Z, A0)
    Fd = api.DeviceFactors.from_numpy(C, F)
    api.cp_als_sweep(C, Zd, Ad, Fd, 3, api.CP_SOLVE_GS, 10, False, api.CP_FP64, None)
    sync()
    A = A0
    for _ in range(3):
        A = amg.bngs(Z, A, F, gs_iters=10, normalize_after=False)
    got = Ad.to_numpy()
    for n in range(3):
        assert elem_err(got[n], A[n]) < 1e-10, (n, elem_err(got[n], A[n]))


@pytest.mark.parametrize("dims,R,sweeps,mixed", [
    ((14, 15, 16), 3, 3, False), ((10, 10, 10), 5, 50, False), ((6, 7, 8, 5), 4, 4, False),
    ((12, 9), 2, 5, False), ((16, 16, 16), 16, 3, False), ((16, 16, 16), 5, 20, True),
    ((7, 5, 9), 8, 6, False), ((40, 70, 3), 4, 4, False), ((130, 6, 5), 3, 4, False)])
def test_small_level_relaxation_matches_oracle(C, dims, R, sweeps, mixed):
    """BNGS sweeps with a right-hand side and Gauss-Seidel solves, no
    normalization (a coarse-level relaxation of Algorithm 2) on tensors that fit
    in LDS: one workgroup runs every sweep.  The shapes cover one and several
    16-row tiles of mode 0 (the matrix-core contractions split over the waves
    or looping over tiles), Grams of more than 64 rows (split over the waves),
    orders 2, 3 and 4, and ragged sizes.  With an FP32 tensor the kernel widens
    each entry and computes in FP64, so it is held against the oracle on the
    FP32-rounded tensor.  The same call with the option off (general kernels)
    agrees too."""
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_OPT_SMALL_LEVELS
    say(f"small-level relaxation dims={dims} R={R} sweeps={sweeps} mixed={mixed}")
    Z, _ = synth.collinear_tensor(dims, min(R, 3), 0.6, 0.02, 0.0, seed=sum(dims))
    A0 = synth.uniform_start(dims, R, 7)
    rng = np.random.default_rng(11)
    F = [0.1 * rng.standard_normal((d, R)) for d in dims]
    Zref = Z.astype(np.float32).astype(np.float64) if mixed else Z
    ref = A0
    for _ in range(sweeps):
        ref = amg.bngs(Zref, ref, F, gs_iters=10, normalize_after=False)
    Fd = api.DeviceFactors.from_numpy(C, F)
    prec = api.CP_MIXED if mixed else api.CP_FP64
    for small in (1, 0):
        C.set_option(CP_OPT_SMALL_LEVELS, small)
        Zd, Ad = dev_inputs(C, Z, A0, fp32=mixed)
        api.cp_als_sweep(C, Zd, Ad, Fd, sweeps, api.CP_SOLVE_GS, 10, False, prec, None)
        sync()
        got = Ad.to_numpy()
        tol = 1e-9 if small else (2e-4 if mixed else 1e-9)
        for n in range(len(dims)):
            e = elem_err(got[n], ref[n], floor=1e-3 if sweeps <= 6 else 1.0)
            assert e < tol, (small, n, e)
    C.set_option(CP_OPT_SMALL_LEVELS, 1)
    assert C.status() == 0


@pytest.mark.parametrize("sweeps", [1, 3])
def test_small_level_gs_zero_pivot_keeps_the_entry(C, sweeps):
    """A zero column in the starting A^(1) makes Gamma^(0) and Gamma^(2) singular
    with a zero diagonal entry: Gauss-Seidel leaves that component of the row as
    it is (Section 5.2 solves only where the pivot is nonzero; the oracle does
    the same), in the small-level kernel and in the general kernels alike."""
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_OPT_SMALL_LEVELS
    say(f"small-level GS zero pivot sweeps={sweeps}")
    dims, R = (10, 11, 12), 3
    rng = np.random.default_rng(8)
    Z = rng.standard_normal(dims)
    A0 = [rng.random((d, R)) for d in dims]
    A0[1][:, 2] = 0.0
    F = [0.1 * rng.standard_normal((d, R)) for d in dims]
    ref = A0
    for _ in range(sweeps):
        ref = amg.bngs(Z, ref, F, gs_iters=10, normalize_after=False)
    Fd = api.DeviceFactors.from_numpy(C, F)
    for small in (1, 0):
        C.set_option(CP_OPT_SMALL_LEVELS, small)
        Zd, Ad = dev_inputs(C, Z, A0, fp32=False)
        api.cp_als_sweep(C, Zd, Ad, Fd, sweeps, api.CP_SOLVE_GS, 10, False, api.CP_FP64, None)
        sync()
        got = Ad.to_numpy()
        for n in range(3):
            e = elem_err(got[n], ref[n], floor=1e-3)
            assert e < 1e-9, (small, n, e)
        if sweeps == 1:
            # mode 0 ran with the zero pivot: column 2 of A^(0) is the start's
            np.testing.assert_array_equal(got[0][:, 2], A0[0][:, 2])
    C.set_option(CP_OPT_SMALL_LEVELS, 1)
    assert C.status() == 0


def test_singular_gamma_uses_pseudoinverse(C):
    from paper_1111_6091_amd import api
    say("pinv fallback")
    dims, R = (10, 11, 12), 3
    rng = np.random.default_rng(6)
    Z = rng.standard_normal(dims)
    A0 = [rng.random((d, R)) for d in dims]
    A0[1][:, 2] = 0.0   # zero column: Gamma^(0) and Gamma^(2) are singular
    Zd, Ad = dev_inputs(C, Z, A0)
    api.cp_als_sweep(C, Zd, Ad, None, 1, api.CP_SOLVE_CHOL, 10, False, api.CP_FP64, None)
    sync()
    flags = C.status()
    from paper_1111_6091_amd import CP_FLAG_PINV_FALLBACK
    assert flags & CP_FLAG_PINV_FALLBACK
    ref = cp.als_sweep(Z, A0, normalize_after=False)
    got = Ad.to_numpy()
    for n in range(3):
        assert elem_err(got[n], ref[n]) < 1e-9, (n, elem_err(got[n], ref[n]))


def test_sort_components(C):
    from paper_1111_6091_amd import api
    rng = np.random.default_rng(8)
    A0 = [rng.standard_normal((d, 5)) for d in (6, 7, 8)]
    A0[0][:, 3] *= 10
    Ad = api.DeviceFactors.from_numpy(C, A0)
    api.cp_sort(C, Ad)
    sync()
    ref, _ = cp.sort_components(A0)
    for g, r in zip(Ad.to_numpy(), ref):
        np.testing.assert_array_equal(g, r)


@pytest.mark.parametrize("I", [20, 21, 128, 7])
def test_transfer_build_matches_oracle(C, I):
    from paper_1111_6091_amd import api
    rng = np.random.default_rng(I)
    w = np.zeros((I, 2))
    for i in range(1, I, 2):
        w[i] = rng.uniform(0.1, 0.9, 2)
        if i + 1 >= I:
            w[i, 1] = 0.0
    wd = torch.from_numpy(w).cuda()
    Ic = (I + 1) // 2
    ph = torch.zeros((I, Ic), dtype=torch.float64, device="cuda")
    api.cp_transfer_build(C, wd, ph)
    sync()
    ref = amg.transfer(amg.interp_from_weights(I, w))[2]
    assert elem_err(ph.cpu().numpy(), ref) < 1e-13


@pytest.mark.parametrize("dims,mask", [((20, 20, 20), (1, 1, 1)), ((17, 12, 9), (1, 0, 1)),
                                       ((16, 18, 10, 12), (1, 1, 1, 1)), ((33, 65, 40), (0, 1, 1))])
def test_restrict_matches_oracle(C, dims, mask):
    from paper_1111_6091_amd import api
    say(f"restrict dims={dims} mask={mask}")
    rng = np.random.default_rng(sum(dims))
    Z = rng.standard_normal(dims)
    phs, phd = [], []
    for d, m in zip(dims, mask):
        if not m:
            phs.append(None)
            phd.append(None)
            continue
        p = amg.transfer(amg.interp_from_weights(d, synth.linear_interp_weights(d)))[2]
        phs.append(p)
        phd.append(torch.from_numpy(p).cuda())
    ref = amg.restrict_tensor(Z, [None if p is None else p.T for p in phs])
    Zd = api.DeviceTensor.from_numpy(C, Z, fp32=True)
    Zc = api.DeviceTensor.empty(ref.shape, fp64=True, fp32=True)
    api.cp_restrict(C, Zd, phd, Zc, api.CP_FP64)
    api.cp_restrict(C, Zd, phd, Zc, api.CP_MIXED)
    sync()
    # error of each entry against the size of the sum it is: the restriction of |Z| by |P^|
    scale = amg.restrict_tensor(np.abs(Z), [None if p is None else np.abs(p.T) for p in phs])
    assert scaled_err(Zc.to_numpy("z64"), ref, scale) < 1e-13
    assert scaled_err(Zc.to_numpy("z32"), ref, scale) < 1e-5


@pytest.mark.parametrize("dims,mask", [((20, 20, 20), (1, 1, 1)), ((17, 12, 9), (1, 0, 1)),
                                       ((16, 18, 10, 12), (1, 1, 1, 1)), ((33, 65, 40), (0, 1, 1)),
                                       ((300, 7, 9), (1, 1, 0)), ((5, 520, 3), (1, 1, 1)), ((2, 3), (1, 1))])
def test_restrict_factored_matches_oracle(C, dims, mask):
    """Eq. (15) in factored form (stencil P^T, then forward substitution with the
    bidiagonal L) against the oracle's mode products with the dense P^, for
    adaptive-looking weights (linear weights scaled at random), FP64 and the FP32
    storage of the mixed form; extents above 128 cross the four-segment blocks."""
    from paper_1111_6091_amd import api
    say(f"factored restrict dims={dims} mask={mask}")
    rng = np.random.default_rng(sum(dims) + 5)
    Z = rng.standard_normal(dims)
    ws, phs = [], []
    for d, m in zip(dims, mask):
        if not m:
            ws.append(None)
            phs.append(None)
            continue
        w = synth.linear_interp_weights(d) * rng.uniform(0.5, 1.5, size=(d, 2))
        w[0::2] = 0.0
        ws.append(w)
        phs.append(amg.transfer(amg.interp_from_weights(d, w))[2])
    ref = amg.restrict_tensor(Z, [None if p is None else p.T for p in phs])
    scale = amg.restrict_tensor(np.abs(Z), [None if p is None else np.abs(p.T) for p in phs])
    wd = [None if w is None else torch.from_numpy(w).cuda() for w in ws]
    Zd = api.DeviceTensor.from_numpy(C, Z, fp32=True)
    Zc = api.DeviceTensor.empty(ref.shape, fp64=True, fp32=True)
    api.cp_restrict_factored(C, Zd, wd, Zc, api.CP_FP64)
    api.cp_restrict_factored(C, Zd, wd, Zc, api.CP_MIXED)
    sync()
    assert scaled_err(Zc.to_numpy("z64"), ref, scale) < 1e-13
    # FP32 storage of input and output, FP64 arithmetic: two roundings to FP32
    Z32 = Z.astype(np.float32).astype(np.float64)
    ref32 = amg.restrict_tensor(Z32, [None if p is None else p.T for p in phs])
    assert scaled_err(Zc.to_numpy("z32"), ref32, scale) < 2e-7
    # the dense form of the same operator agrees
    phd = [None if p is None else torch.from_numpy(p).cuda() for p in phs]
    Zg = api.DeviceTensor.empty(ref.shape)
    api.cp_restrict(C, Zd, phd, Zg, api.CP_FP64)
    sync()
    assert scaled_err(Zc.to_numpy("z64"), Zg.to_numpy(), scale) < 1e-13
    assert C.status() == 0


def test_identity_restriction_returns_z(C):
    from paper_1111_6091_amd import api
    Z = np.random.default_rng(1).standard_normal((5, 6, 7))
    Zd = api.DeviceTensor.from_numpy(C, Z)
    Zc = api.DeviceTensor.empty(Z.shape)
    api.cp_restrict(C, Zd, [None, None, None], Zc)
    sync()
    np.testing.assert_array_equal(Zc.to_numpy(), Z)


@pytest.mark.parametrize("I,R", [(21, 4), (130, 5), (3, 1)])
def test_prolong_and_restrict_factor(C, I, R):
    """A = P^ Ac, A += P^ (Ac - A~c) and A~c = P^T A (Algorithm 2's transfers of
    the factors): sizes whose contraction is shorter than, a ragged multiple of,
    and several times the kernels' eight-lane split."""
    from paper_1111_6091_amd import api
    rng = np.random.default_rng(9)
    p = amg.transfer(amg.interp_from_weights(I, synth.linear_interp_weights(I)))[2]
    Ic = p.shape[1]
    A = rng.standard_normal((I, R))
    Ac = rng.standard_normal((Ic, R))
    Act = rng.standard_normal((Ic, R))
    pd = torch.from_numpy(p).cuda()
    Ad = torch.from_numpy(A.copy()).cuda()
    out = torch.zeros((Ic, R), dtype=torch.float64, device="cuda")
    api.cp_restrict_factor(C, pd, Ad, out)
    sync()
    assert scaled_err(out.cpu().numpy(), p.T @ A, np.abs(p.T) @ np.abs(A)) < 1e-14
    api.cp_prolong(C, pd, torch.from_numpy(Ac).cuda(), torch.from_numpy(Act).cuda(), Ad)
    sync()
    assert scaled_err(Ad.cpu().numpy(), A + p @ (Ac - Act), np.abs(A) + np.abs(p) @ (np.abs(Ac) + np.abs(Act))) < 1e-14
    api.cp_prolong(C, pd, torch.from_numpy(Ac).cuda(), None, Ad)
    sync()
    assert scaled_err(Ad.cpu().numpy(), p @ Ac, np.abs(p) @ np.abs(Ac)) < 1e-14


def _oracle_levels(Z, weights, coarsest):
    return amg.hierarchy_from_weights(Z, weights, coarsest)


@pytest.mark.parametrize("small", [1, 0])
@pytest.mark.parametrize("dims,R,nlev", [((20, 20, 20), 3, 2), ((32, 32, 32), 3, 3), ((24, 20, 6), 2, 2)])
def test_fas_vcycle_matches_oracle(C, dims, R, nlev, small):
    from paper_1111_6091_amd import api, drivers
    from paper_1111_6091_amd._lib import CP_OPT_SMALL_LEVELS
    C.set_option(CP_OPT_SMALL_LEVELS, small)
    say(f"fas vcycle dims={dims} R={R} levels={nlev} small-level kernel={small}")
    Z, _ = synth.collinear_tensor(dims, R, 0.5, 0.01, 0.0, seed=10)
    A0, _ = cp.als(Z, synth.uniform_start(dims, R, 10), max_sweeps=10, fit_tol=0.0, sort_at_end=False)
    # weights per level (linear interpolation); modes of size <= 6 are not coarsened
    weights, cur = [], list(dims)
    coarsest = [max(6, R)] * len(dims)
    for _ in range(nlev - 1):
        wl = [synth.linear_interp_weights(d) if d > coarsest[n] else None for n, d in enumerate(cur)]
        weights.append(wl)
        cur = [(d + 1) // 2 if wl[n] is not None else d for n, d in enumerate(cur)]
    levels = _oracle_levels(Z, weights, coarsest)
    assert len(levels) == nlev
    ref = amg.fas_vcycle(levels, amg.zeros_like_factors(A0), A0, nu1=1, nu2=1, nuc=20)
    Zd = api.DeviceTensor.from_numpy(C, Z)
    dlev = drivers.build_hierarchy(C, Zd, weights)
    Ad = api.DeviceFactors.from_numpy(C, A0)
    api.cp_fas_vcycle(C, dlev, Ad, nu1=1, nu2=1, nuc=20)
    sync()
    got = Ad.to_numpy()
    for n in range(len(dims)):
        assert elem_err(got[n], ref[n]) < 1e-9, (n, elem_err(got[n], ref[n]))
    assert elem_err(cp.full(got), cp.full(ref)) < 1e-11
    C.set_option(CP_OPT_SMALL_LEVELS, 1)

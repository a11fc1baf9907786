"""Edge cases of the C ABI against the oracle: the largest rank and order the
library takes, order-2 tensors, rank one, modes of extent one, rank above a
mode's extent, and argument errors caught on the host before any launch."""
import numpy as np
import pytest

from oracle import cp
from paper_1111_6091_amd import synth
from tests.gpu_util import ctx as make_ctx, elem_err, mttkrp_err, say, sync

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def C():
    return make_ctx()


def _inputs(C, dims, R, seed, fp32=False):
    from paper_1111_6091_amd import api
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal(dims)
    A = [rng.random((d, R)) for d in dims]
    return Z, A, api.DeviceTensor.from_numpy(C, Z, fp32=fp32), api.DeviceFactors.from_numpy(C, A, fp32=fp32)


EDGE_SHAPES = [
    ((6, 5, 4), 32),                    # maximum rank (two 16-column tiles), R > every extent
    ((3, 2, 2, 3, 2, 2, 3, 2), 4),      # maximum order, 6 stripe modes
    ((33, 17), 5),                      # order 2 (no stripe modes)
    ((9, 1, 7), 3),                     # a mode of extent one
    ((1, 12, 10), 2),                   # contiguous extent one
    ((40, 30, 20), 1),                  # rank one
]


@pytest.mark.parametrize("dims,R", EDGE_SHAPES)
@pytest.mark.parametrize("mixed", [False, True])
def test_mttkrp_edge_shapes(C, dims, R, mixed):
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED
    say(f"edge mttkrp dims={dims} R={R} mixed={mixed}")
    Z, A, Zd, Ad = _inputs(C, dims, R, 7, fp32=mixed)
    for n in range(len(dims)):
        M = torch.empty((dims[n], R), dtype=torch.float64, device="cuda")
        api.cp_mttkrp(C, Zd, Ad, n, M, CP_MIXED if mixed else CP_FP64)
        sync()
        e = mttkrp_err(M.cpu().numpy(), Z, A, n)
        assert e < (2e-5 if mixed else 1e-12), (n, e)


@pytest.mark.parametrize("dims,R", [((40, 36, 6), 32), ((3, 2, 2, 3, 2, 2, 3, 2), 4), ((33, 17), 5),
                                    ((9, 1, 7), 3), ((40, 30, 20), 1)])
def test_als_sweeps_edge_shapes(C, dims, R):
    """Three sweeps against the oracle.  Each shape keeps every Gamma^(n) positive
    definite (some other mode has extent >= R, or the Hadamard product of the
    lower-rank Grams is generically full rank), so the Cholesky path is taken and
    the factors are unique; the singular case has its own test."""
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_FP64, CP_SOLVE_CHOL
    say(f"edge sweeps dims={dims} R={R}")
    if min(dims) >= 3:
        Z, _ = synth.collinear_tensor(dims, 3, 0.5, 0.01, 0.0, seed=3)
    else:
        Z = np.random.default_rng(3).standard_normal(dims)
    A0 = synth.uniform_start(dims, R, 3)
    Zd = api.DeviceTensor.from_numpy(C, Z)
    Ad = api.DeviceFactors.from_numpy(C, A0)
    api.cp_als_sweep(C, Zd, Ad, None, 3, CP_SOLVE_CHOL, 10, True, CP_FP64)
    sync()
    ref = [a.copy() for a in A0]
    for _ in range(3):
        ref = cp.als_sweep(Z, ref)
    got = Ad.to_numpy()
    assert C.status() == 0
    # at R = 32 Gamma has a condition number near 2e6, so each solve carries
    # absolute errors of about cond(Gamma) u max|A| (1e-10 max|A|) into entries
    # of any size: there every entry is held against the factor's largest one
    fl = 1.0 if R >= 32 else 1e-3
    for n in range(len(dims)):
        assert elem_err(got[n], ref[n], floor=fl) < 1e-8, (n, elem_err(got[n], ref[n], floor=fl))
    assert elem_err(cp.full(got), cp.full(ref), floor=fl) < 1e-9


def test_host_side_argument_errors(C):
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_ERR_INVALID, CP_ERR_SHAPE, CP_FP64
    Z, A, Zd, Ad = _inputs(C, (5, 6, 7), 3, 1)
    M = torch.empty((5, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(api.CpError) as e:
        api.cp_mttkrp(C, Zd, Ad, 3, M, CP_FP64)        # mode out of range
    assert e.value.code == CP_ERR_INVALID
    with pytest.raises(api.CpError):
        api.cp_mttkrp(C, Zd, Ad, 0, M, 1)              # mixed without FP32 shadows
    bad = api.DeviceTensor((5, 0, 7), z64=Zd.z64, norm2=Zd.norm2)
    with pytest.raises(api.CpError) as e:
        api.cp_mttkrp(C, bad, Ad, 0, M, CP_FP64)       # empty mode
    assert e.value.code == CP_ERR_SHAPE
    big = api.DeviceFactors([torch.zeros((d, 33), dtype=torch.float64, device="cuda") for d in (5, 6, 7)])
    with pytest.raises(api.CpError) as e:
        api.cp_als_sweep(C, Zd, big, None, 1)          # rank above the maximum
    assert e.value.code == CP_ERR_SHAPE
    with pytest.raises(api.CpError):
        api.cp_als_sweep(C, Zd, Ad, None, -1)          # negative sweep count
    assert C.status() == 0


@pytest.mark.parametrize("R", [14, 20, 32])
def test_als_sweeps_dimension_tree_wide_rank(C, R):
    """Three FP64 sweeps at 128 x 12 x 12 with R = 14, 20, 32: the dimension
    tree applies (Y is a quarter of Z), so mode 2 runs the Y-contracting kernel,
    whose bookkeeping factors Gamma with 16-, 24- and 32-entry register rows."""
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_FP64, CP_SOLVE_CHOL
    dims = (128, 12, 12)
    say(f"dimension-tree sweeps dims={dims} R={R}")
    Z, _ = synth.collinear_tensor(dims, 3, 0.5, 0.01, 0.0, seed=3)
    A0 = synth.uniform_start(dims, R, 3)
    Zd = api.DeviceTensor.from_numpy(C, Z)
    Ad = api.DeviceFactors.from_numpy(C, A0)
    K = 3
    fh = torch.zeros(K, dtype=torch.float64, device="cuda")
    api.cp_als_sweep(C, Zd, Ad, None, K, CP_SOLVE_CHOL, 10, True, CP_FP64, fh)
    sync()
    assert C.status() == 0
    ref = [a.copy() for a in A0]
    fref = []
    for _ in range(K):
        ref = cp.als_sweep(Z, ref)
        fref.append(cp.objective(Z, ref))
    got = Ad.to_numpy()
    # at R = 32 against the factor's largest entry (Gamma's condition number grows with R)
    fl = 1.0 if R >= 32 else 1e-3
    for n in range(3):
        assert elem_err(got[n], ref[n], floor=fl) < 1e-8, (n, elem_err(got[n], ref[n], floor=fl))
    np.testing.assert_allclose(fh.cpu().numpy(), fref, rtol=1e-9)

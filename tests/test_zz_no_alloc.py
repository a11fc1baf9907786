"""The allocation-free MTTKRP entry point against cp_mttkrp, through the C ABI.

cp_mttkrp_noalloc runs the same launch configuration and kernels as cp_mttkrp
with its partial sums in the library's static scratch array, so the two agree
bit for bit.  Two calls in a row, the second on a smaller tensor, check that
the shared scratch carries nothing over between calls; a fresh context checks
that no device memory is allocated on the way.
"""
import numpy as np
import pytest

from paper_1111_6091_amd import synth
from tests.gpu_util import ctx as make_ctx, have_gpu, mttkrp_err, say, sync

pytestmark = pytest.mark.gpu


def _problem(C, dims, R, seed, fp32):
    from paper_1111_6091_amd import api
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal(dims)
    A = [rng.uniform(size=(d, R)) for d in dims]
    return Z, A, api.DeviceTensor.from_numpy(C, Z, fp32=fp32), api.DeviceFactors.from_numpy(C, A, fp32=fp32)


@pytest.mark.parametrize("mixed", [False, True])
def test_noalloc_matches_cp_mttkrp_on_two_calls(mixed):
    import torch
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_FP64, CP_MIXED
    if not have_gpu():
        pytest.skip("no GPU")
    prec = CP_MIXED if mixed else CP_FP64
    C = make_ctx()
    # a large case (split contractions: partials in the scratch array), then a smaller one
    cases = [((96, 80, 72), 10, 11), ((40, 36, 30, 5), 7, 12)]
    for dims, R, seed in cases:
        say(f"noalloc mixed={mixed} dims={dims} R={R}")
        Z, A, Zd, Ad = _problem(C, dims, R, seed, mixed)
        for n in range(len(dims)):
            M1 = torch.full((dims[n], R), np.nan, dtype=torch.float64, device="cuda")
            M2 = torch.full((dims[n], R), np.nan, dtype=torch.float64, device="cuda")
            api.cp_mttkrp_noalloc(C, Zd, Ad, n, M1, prec)
            api.cp_mttkrp(C, Zd, Ad, n, M2, prec)
            sync()
            a, b = M1.cpu().numpy(), M2.cpu().numpy()
            assert np.array_equal(a, b), (dims, n, np.max(np.abs(a - b)))
            err = mttkrp_err(a, Z, A, n)
            assert err < (2e-5 if mixed else 1e-12), (dims, n, err)
    assert C.status() == 0


def test_noalloc_allocates_no_device_memory():
    import torch
    from paper_1111_6091_amd import api
    from paper_1111_6091_amd._lib import CP_FP64
    if not have_gpu():
        pytest.skip("no GPU")
    C = make_ctx()   # fresh context: empty workspace
    dims, R = (128, 96, 64), 8
    Z, A, Zd, Ad = _problem(C, dims, R, 13, False)
    Ms = [torch.empty((d, R), dtype=torch.float64, device="cuda") for d in dims]
    sync()
    free0, _ = torch.cuda.mem_get_info()
    for n in range(3):
        api.cp_mttkrp_noalloc(C, Zd, Ad, n, Ms[n], CP_FP64)
    sync()
    free1, _ = torch.cuda.mem_get_info()
    say(f"free device memory before {free0}, after {free1}")
    # the context's workspace is at least 1 MiB when it is first allocated
    assert free0 - free1 < (1 << 20)
    for n in range(3):
        assert mttkrp_err(Ms[n].cpu().numpy(), Z, A, n) < 1e-12, n

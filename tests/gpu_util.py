"""Helpers shared by the GPU parity tests (test infrastructure)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def ctx():
    from paper_1111_6091_amd import api
    return api.Context()


def sync():
    import torch
    torch.cuda.synchronize()


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm((a - b).ravel())
    n = np.linalg.norm(b.ravel())
    return d / n if n > 0 else d


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def elem_err(a, b, floor=1e-3):
    """max_i |a_i - b_i| / (|b_i| + floor * max|b|): element by element, with a
    floor for entries far below the largest one."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.size == 0:
        return 0.0
    den = np.abs(b) + floor * np.max(np.abs(b))
    den = np.where(den > 0, den, 1.0)
    return float(np.max(np.abs(a - b) / den))


def mttkrp_err(got, Z, A, n):
    """Element-wise error of an MTTKRP result against the oracle, relative to the
    scale a floating-point sum of its terms is accurate to: the MTTKRP of |Z|
    with |A^(m)|, i.e. sum over the contraction of |z| prod |a|.  A summation of
    K terms in precision u is within about K u of it per element (FP32 GEMM
    chunks of K <= 256: about 1.5e-5; FP64: below 1e-12)."""
    from oracle import cp
    ref = cp.mttkrp(Z, A, n)
    scale = cp.mttkrp(np.abs(Z), [np.abs(a) for a in A], n)
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(np.asarray(got, dtype=np.float64) - ref) / scale))


def scaled_err(got, ref, scale):
    """max_i |got_i - ref_i| / scale_i, where scale_i is the sum of the absolute
    values of the terms that make ref_i (what a floating-point sum is accurate to)."""
    scale = np.asarray(scale, dtype=np.float64)
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(np.asarray(got, dtype=np.float64) - np.asarray(ref, dtype=np.float64)) / scale))

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

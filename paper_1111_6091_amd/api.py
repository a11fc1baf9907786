"""Python binding of libcpamg: same call names as the C ABI, argument marshalling only.

PyTorch supplies device memory and the stream; every computation runs in the
HIP kernels of libcpamg.  Device tensors use the library layouts: a tensor is a
1-D buffer with mode 1 fastest; a factor A^(n) is an (I_n, R) row-major tensor.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as L
from ._lib import (CP_FP64, CP_MIXED, CP_SOLVE_CHOL, CP_SOLVE_GS, CpBatchParams, CpBatchProblem,
                   CpFactors, CpFasParams, CpLevel, CpTensor)


class CpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libcpamg error {code}: {msg}")
        self.code = code


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else int(t.data_ptr()))


class Context:
    """A libcpamg context bound to a HIP stream (default: torch's current stream)."""

    def __init__(self, stream=None):
        torch = _torch()
        self._lib = L.load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self._lib.cp_ctx_create(ctypes.byref(h), ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise CpError(rc, "cp_ctx_create failed")
        self.handle = h

    def check(self, rc):
        if rc != 0:
            msg = self._lib.cp_last_error(self.handle)
            raise CpError(rc, msg.decode() if msg else "")

    def status(self):
        flags = ctypes.c_int32(0)
        self.check(self._lib.cp_get_status(self.handle, ctypes.byref(flags)))
        return flags.value

    def set_option(self, option, value):
        self.check(self._lib.cp_set_option(self.handle, int(option), int(value)))

    def profile(self, on=True):
        self.check(self._lib.cp_profile_enable(self.handle, int(bool(on))))

    def profile_read(self):
        n = len(L.PROF_CLASSES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int32 * n)()
        self.check(self._lib.cp_profile_read(self.handle, ms, cnt))
        return {L.PROF_CLASSES[k]: (ms[k], cnt[k]) for k in range(n) if cnt[k]}

    def close(self):
        if getattr(self, "handle", None):
            self._lib.cp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceTensor:
    """Dense tensor in device memory (mode 1 fastest), FP64 master + optional FP32 shadow."""

    def __init__(self, dims, z64=None, z32=None, norm2=None):
        self.dims = tuple(int(d) for d in dims)
        self.z64, self.z32, self.norm2 = z64, z32, norm2

    @property
    def order(self):
        return len(self.dims)

    @property
    def numel(self):
        return int(np.prod(self.dims))

    @property
    def device(self):
        return (self.z64 if self.z64 is not None else self.z32).device

    @classmethod
    def from_numpy(cls, ctx, Z, fp32=False, device="cuda"):
        torch = _torch()
        Z = np.asarray(Z, dtype=np.float64)
        z64 = torch.from_numpy(np.ascontiguousarray(Z.ravel(order="F"))).to(device)
        t = cls(Z.shape, z64=z64)
        t.norm2 = torch.zeros(1, dtype=torch.float64, device=device)
        cp_norm2(ctx, t, t.norm2)
        if fp32:
            t.z32 = torch.empty(t.numel, dtype=torch.float32, device=device)
            cp_cast_f32(ctx, t.z64, t.z32)
        return t

    @classmethod
    def empty(cls, dims, fp64=True, fp32=False, device="cuda"):
        torch = _torch()
        P = int(np.prod(dims))
        return cls(dims, z64=torch.empty(P, dtype=torch.float64, device=device) if fp64 else None,
                   z32=torch.empty(P, dtype=torch.float32, device=device) if fp32 else None)

    def struct(self):
        s = CpTensor()
        s.order = self.order
        for i, d in enumerate(self.dims):
            s.dims[i] = d
        s.z64 = _ptr(self.z64).value
        s.z32 = _ptr(self.z32).value
        s.norm2 = _ptr(self.norm2).value
        return s

    def to_numpy(self, which="z64"):
        buf = getattr(self, which)
        return buf.detach().cpu().numpy().astype(np.float64).reshape(self.dims, order="F")


class SparseTensor:
    """Sparse tensor in device memory (cp_tensor's sparse form): coordinate
    entries (idx nnz x N int32, vals nnz FP64) and the per-mode orderings that
    cp_sparse_index builds on the host."""

    def __init__(self, dims, idx, vals, rowptr, perm, norm2=None):
        self.dims = tuple(int(d) for d in dims)
        self.idx, self.vals, self.rowptr, self.perm, self.norm2 = idx, vals, rowptr, perm, norm2
        self.z64 = self.z32 = None

    @property
    def order(self):
        return len(self.dims)

    @property
    def nnz(self):
        return int(self.vals.numel())

    @property
    def device(self):
        return self.vals.device

    @classmethod
    def from_coo(cls, ctx, idx, vals, dims, device="cuda"):
        torch = _torch()
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
        vals = np.ascontiguousarray(np.asarray(vals, dtype=np.float64))
        N, nnz = len(dims), vals.shape[0]
        if idx.shape != (nnz, N):
            raise ValueError(f"idx has shape {idx.shape}, expected ({nnz}, {N})")
        dd = (ctypes.c_int64 * N)(*[int(d) for d in dims])
        rowptr = np.zeros(sum(int(d) + 1 for d in dims), dtype=np.int64)
        perm = np.zeros(N * nnz, dtype=np.int32)
        ctx.check(ctx._lib.cp_sparse_index(ctx.handle, N, dd, nnz, idx.ctypes.data_as(ctypes.c_void_p),
                                           rowptr.ctypes.data_as(ctypes.c_void_p),
                                           perm.ctypes.data_as(ctypes.c_void_p)))
        t = cls(dims, torch.from_numpy(idx).to(device), torch.from_numpy(vals).to(device),
                torch.from_numpy(rowptr).to(device), torch.from_numpy(perm).to(device))
        t.norm2 = torch.zeros(1, dtype=torch.float64, device=device)
        cp_norm2(ctx, t, t.norm2)
        return t

    def struct(self):
        s = CpTensor()
        s.order = self.order
        for i, d in enumerate(self.dims):
            s.dims[i] = d
        s.norm2 = _ptr(self.norm2).value
        s.nnz = self.nnz
        s.idx = _ptr(self.idx).value
        s.vals = _ptr(self.vals).value
        rp0, pm0 = int(self.rowptr.data_ptr()), int(self.perm.data_ptr())
        off = 0
        for m, d in enumerate(self.dims):
            s.rowptr[m] = rp0 + 8 * off
            s.perm[m] = pm0 + 4 * m * self.nnz
            off += d + 1
        return s


class DeviceFactors:
    """Kruskal factors: list of (I_n, R) float64 device tensors (+ optional FP32 shadows)."""

    def __init__(self, mats, mats32=None):
        self.mats = list(mats)
        self.mats32 = list(mats32) if mats32 is not None else None

    @property
    def rank(self):
        return int(self.mats[0].shape[1])

    @property
    def dims(self):
        return tuple(int(m.shape[0]) for m in self.mats)

    @classmethod
    def from_numpy(cls, ctx, A, fp32=False, device="cuda"):
        torch = _torch()
        mats = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device) for a in A]
        m32 = None
        if fp32:
            m32 = [torch.empty(m.shape, dtype=torch.float32, device=device) for m in mats]
            for a, b in zip(mats, m32):
                cp_cast_f32(ctx, a, b)
        return cls(mats, m32)

    @classmethod
    def zeros(cls, dims, R, fp32=False, device="cuda"):
        torch = _torch()
        mats = [torch.zeros((d, R), dtype=torch.float64, device=device) for d in dims]
        m32 = [torch.zeros((d, R), dtype=torch.float32, device=device) for d in dims] if fp32 else None
        return cls(mats, m32)

    def clone(self):
        return DeviceFactors([m.clone() for m in self.mats],
                             [m.clone() for m in self.mats32] if self.mats32 else None)

    def struct(self):
        s = CpFactors()
        s.rank = self.rank
        for i, m in enumerate(self.mats):
            s.a[i] = int(m.data_ptr())
            if self.mats32 is not None:
                s.a32[i] = int(self.mats32[i].data_ptr())
        return s

    def to_numpy(self):
        return [m.detach().cpu().numpy().copy() for m in self.mats]


# ---------------------------------------------------------------------------
# calls (same names as the C ABI)
# ---------------------------------------------------------------------------
def cp_cast_f32(ctx, src, dst):
    ctx.check(ctx._lib.cp_cast_f32(ctx.handle, _ptr(src), _ptr(dst), ctypes.c_int64(src.numel())))


def cp_norm2(ctx, Z, out):
    s = Z.struct()
    ctx.check(ctx._lib.cp_norm2(ctx.handle, ctypes.byref(s), _ptr(out)))


def cp_mttkrp(ctx, Z, A, n, M, prec=CP_FP64):
    zs, fs = Z.struct(), A.struct()
    ctx.check(ctx._lib.cp_mttkrp(ctx.handle, ctypes.byref(zs), ctypes.byref(fs), n, _ptr(M), prec))


def cp_mttkrp_noalloc(ctx, Z, A, n, M, prec=CP_FP64):
    zs, fs = Z.struct(), A.struct()
    ctx.check(ctx._lib.cp_mttkrp_noalloc(ctx.handle, ctypes.byref(zs), ctypes.byref(fs), n, _ptr(M),
                                         prec))


def cp_als_sweep(ctx, Z, A, F=None, nsweeps=1, solver=CP_SOLVE_CHOL, gs_iters=10, normalize=True,
                 prec=CP_FP64, f_hist=None):
    zs, fs = Z.struct(), A.struct()
    Fs = F.struct() if F is not None else None
    ctx.check(ctx._lib.cp_als_sweep(ctx.handle, ctypes.byref(zs), ctypes.byref(fs),
                                    ctypes.byref(Fs) if Fs is not None else None, nsweeps, solver,
                                    gs_iters, int(bool(normalize)), prec, _ptr(f_hist)))


def cp_objective(ctx, Z, A, exact=True, f=None, g=None, prec=CP_FP64):
    zs, fs = Z.struct(), A.struct()
    ctx.check(ctx._lib.cp_objective(ctx.handle, ctypes.byref(zs), ctypes.byref(fs), int(bool(exact)),
                                    _ptr(f), _ptr(g), prec))


def _phat_array(phat):
    arr = (ctypes.c_void_p * L.CP_MAX_ORDER)()
    for i, p in enumerate(phat):
        arr[i] = None if p is None else int(p.data_ptr())
    return arr


def cp_restrict(ctx, Z, phat, Zc, prec=CP_FP64):
    zs, cs = Z.struct(), Zc.struct()
    ctx.check(ctx._lib.cp_restrict(ctx.handle, ctypes.byref(zs), _phat_array(phat), ctypes.byref(cs),
                                   prec))


def cp_restrict_factored(ctx, Z, w, Zc, prec=CP_FP64):
    """w: per mode (I_n x 2) device weights or None (identity)."""
    zs, cs = Z.struct(), Zc.struct()
    ctx.check(ctx._lib.cp_restrict_factored(ctx.handle, ctypes.byref(zs), _phat_array(w), ctypes.byref(cs),
                                            prec))


def cp_prolong(ctx, phat, Ac, Ac_tilde, A):
    I, R = A.shape
    Ic = Ac.shape[0]
    ctx.check(ctx._lib.cp_prolong(ctx.handle, I, Ic, R, _ptr(phat), _ptr(Ac), _ptr(Ac_tilde), _ptr(A)))


def cp_restrict_factor(ctx, phat, A, Ac):
    I, R = A.shape
    Ic = Ac.shape[0]
    ctx.check(ctx._lib.cp_restrict_factor(ctx.handle, I, Ic, R, _ptr(phat), _ptr(A), _ptr(Ac)))


def cp_interp_weights(ctx, Z, A, groups, nfit, n, w):
    zs, fs = Z.struct(), A.struct()
    ctx.check(ctx._lib.cp_interp_weights(ctx.handle, ctypes.byref(zs), ctypes.byref(fs), int(groups),
                                         int(nfit), int(n), _ptr(w)))


def cp_transfer_build(ctx, w, phat):
    I = w.shape[0]
    ctx.check(ctx._lib.cp_transfer_build(ctx.handle, I, _ptr(w), _ptr(phat)))


def cp_fas_vcycle(ctx, levels, A, nu1=1, nu2=1, nuc=50, gs_iters=10, ic_rule=0, prec=CP_FP64):
    """levels: list of (DeviceTensor, [phat_n or None per mode]) from finest to coarsest."""
    arr = (CpLevel * len(levels))()
    for i, (Zl, ph) in enumerate(levels):
        arr[i].z = Zl.struct()
        for n in range(L.CP_MAX_ORDER):
            p = ph[n] if ph is not None and n < len(ph) else None
            arr[i].phat[n] = None if p is None else int(p.data_ptr())
    prm = CpFasParams(nu1, nu2, nuc, gs_iters, ic_rule)
    fs = A.struct()
    ctx.check(ctx._lib.cp_fas_vcycle(ctx.handle, arr, len(levels), ctypes.byref(fs),
                                     ctypes.byref(prm), prec))


def cp_time_mttkrp(ctx, Z, A, n, prec=CP_FP64, reps=20):
    zs, fs = Z.struct(), A.struct()
    ms = ctypes.c_double(0.0)
    ctx.check(ctx._lib.cp_time_mttkrp(ctx.handle, ctypes.byref(zs), ctypes.byref(fs), n, prec, reps,
                                      ctypes.byref(ms)))
    return ms.value


def cp_autotune(ctx, Z, A, prec=CP_FP64, reps=20):
    zs, fs = Z.struct(), A.struct()
    ctx.check(ctx._lib.cp_autotune(ctx.handle, ctypes.byref(zs), ctypes.byref(fs), prec, reps))


def cp_plans_export(ctx):
    return ctx._lib.cp_plans_export(ctx.handle).decode()


def cp_plans_import(ctx, text):
    ctx.check(ctx._lib.cp_plans_import(ctx.handle, text.encode()))


def cp_sort(ctx, A):
    dims = (ctypes.c_int64 * L.CP_MAX_ORDER)(*A.dims)
    fs = A.struct()
    ctx.check(ctx._lib.cp_sort(ctx.handle, dims, len(A.mats), ctypes.byref(fs)))


def cp_als_batched(ctx, problems, restarts, prec=CP_MIXED, window32=16, tol32=1e-9, tol64=1e-12,
                   max_sweeps=10000, chunk=16, wg_kib=0):
    """Batched ALS solves: ``problems`` is a list of (DeviceTensor, DeviceFactors) where the
    factors have rank restarts * R (restart k in columns k*R..(k+1)*R-1).  Returns device
    tensors (fits [nprob, restarts], sweeps [nprob, restarts, 2])."""
    torch = _torch()
    n = len(problems)
    arr = (CpBatchProblem * n)()
    for i, (Z, A) in enumerate(problems):
        arr[i].z = Z.struct()
        arr[i].a = A.struct()
    prm = CpBatchParams(restarts, prec, window32, tol32, tol64, max_sweeps, chunk, wg_kib)
    dev = problems[0][0].z64.device
    fits = torch.empty((n, restarts), dtype=torch.float64, device=dev)
    sweeps = torch.empty((n, restarts, 2), dtype=torch.int32, device=dev)
    ctx.check(ctx._lib.cp_als_batched(ctx.handle, arr, n, ctypes.byref(prm), _ptr(fits), _ptr(sweeps)))
    return fits, sweeps

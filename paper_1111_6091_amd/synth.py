"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws random numbers and assembles test tensors.  It holds none
of the decomposition method's arithmetic (no MTTKRP, no Gram/Hadamard products,
no solves, no transfer operators) and imports neither the oracle nor the HIP
binding, so both sides can take their inputs from it without sharing code.

Collinear-factor design (used for every synthetic workload):

1. for every mode n: G_n ~ N(0,1)^{I_n x R}; Q_n is the thin QR factor of G_n
   with column signs chosen so that diag(R_qr) > 0; C = (1-c) I + c 11^T,
   U = upper Cholesky factor of C (C = U^T U); A_n = sqrt(I_n) Q_n U, so that
   A_n^T A_n = I_n C: every pair of columns has cosine exactly c;
2. T = sum_r a_r^(1) o ... o a_r^(N)  (mode 1 fastest in memory);
3. E1 ~ N(0,1), Z = T + eta_h ||T|| E1/||E1||   (homoscedastic noise);
4. if eta_x > 0: E2 = N(0,1) * T (entrywise), Z += eta_x ||T|| E2/||E2||
   (heteroscedastic noise);
5. a random start for restart k is drawn from default_rng(seed + 1 + k) as
   U(0,1) entries (the initial guesses of the paper's experiments are uniform).

All draws come from one numpy ``default_rng(seed)`` (PCG64) in the order above.
Tensors are returned as numpy arrays of logical shape (I_1, ..., I_N) stored in
Fortran order (mode 1 fastest), which is also the device layout.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "collinear_factors", "outer_sum", "collinear_tensor", "uniform_start",
    "linear_interp_weights", "WORKLOADS", "workload", "batched_problems",
    "dense_ijk", "DENSE_TESTS", "dense_case", "dense_coarse_start",
    "laplacian_coo", "coo_to_dense", "LAPLACIAN_TESTS", "LAPLACIAN_COARSEST", "laplacian_case",
]


def collinear_factors(rng: np.random.Generator, dims, R: int, c: float):
    """Draw N factor matrices (I_n x R, C-contiguous) with pairwise column cosine c."""
    C = (1.0 - c) * np.eye(R) + c * np.ones((R, R))
    U = np.linalg.cholesky(C).T          # upper factor, C = U^T U
    out = []
    for In in dims:
        if In < R:
            raise ValueError(f"mode size {In} < rank {R}: columns cannot be made collinear")
        G = rng.standard_normal((In, R))
        Q, Rq = np.linalg.qr(G)
        s = np.sign(np.diag(Rq))
        s[s == 0] = 1.0
        Q = Q * s
        out.append(np.ascontiguousarray(np.sqrt(In) * (Q @ U)))
    return out


def outer_sum(factors):
    """Assemble sum_r a_r^(1) o ... o a_r^(N) as an F-ordered array (input synthesis only)."""
    N = len(factors)
    letters = "abcdefgh"[:N]
    spec = ",".join(f"{l}z" for l in letters) + "->" + letters
    T = np.einsum(spec, *factors, optimize=True)
    return np.asfortranarray(T)


def _normal_like(rng, shape):
    P = int(np.prod(shape))
    return rng.standard_normal(P).reshape(shape, order="F")


def collinear_tensor(dims, R, c, eta_h, eta_x=0.0, seed=0):
    """Return (Z, true_factors) for the collinear design with the given noise levels."""
    rng = np.random.default_rng(seed)
    A = collinear_factors(rng, dims, R, c)
    T = outer_sum(A)
    nT = np.linalg.norm(T.ravel(order="K"))
    Z = T.copy(order="F")
    if eta_h > 0:
        E1 = _normal_like(rng, dims)
        Z += (eta_h * nT / np.linalg.norm(E1.ravel(order="K"))) * E1
    if eta_x > 0:
        E2 = _normal_like(rng, dims) * T
        Z += (eta_x * nT / np.linalg.norm(E2.ravel(order="K"))) * E2
    return np.asfortranarray(Z), A


def uniform_start(dims, R, seed, restart=0):
    """U(0,1) initial factor matrices for restart ``restart`` (seed + 1 + restart)."""
    rng = np.random.default_rng(seed + 1 + restart)
    return [np.ascontiguousarray(rng.random((In, R))) for In in dims]


def linear_interp_weights(I):
    """Interpolation weights (I x 2) for geometric coarsening with equal weights 1/2.

    Row i (0-based) with i odd is a fine point between coarse points (i-1)/2 and
    (i+1)/2; its weights are (1/2, 1/2), or (1, 0) at a right endpoint with a single
    coarse neighbour.  Rows of coarse points are ignored by the consumer (they are
    injections).  This is a fixed, data-independent input for kernel tests and
    timing; the adaptive least-squares weights are computed elsewhere.
    """
    w = np.zeros((I, 2))
    for i in range(1, I, 2):
        if i + 1 < I:
            w[i] = (0.5, 0.5)
        else:
            w[i] = (1.0, 0.0)
    return w


# Named workloads: dims, rank, collinearity, homoscedastic / heteroscedastic noise, seed.
WORKLOADS = {
    "c1_20cube_r3": dict(dims=(20, 20, 20), R=3, c=0.5, eta_h=0.01, eta_x=0.0, seed=1),
    "c2_128cube_r5": dict(dims=(128, 128, 128), R=5, c=0.9, eta_h=0.01, eta_x=0.01, seed=2),
    "c3_256cube_r10": dict(dims=(256, 256, 256), R=10, c=0.9, eta_h=0.01, eta_x=0.0, seed=3),
    "c4_64quart_r8": dict(dims=(64, 64, 64, 64), R=8, c=0.8, eta_h=0.005, eta_x=0.0, seed=4),
}


def workload(name):
    """Build a named workload: returns (Z, true_factors, spec)."""
    spec = WORKLOADS[name]
    Z, A = collinear_tensor(spec["dims"], spec["R"], spec["c"], spec["eta_h"],
                            spec["eta_x"], spec["seed"])
    return Z, A, spec


def batched_problems(count=512, seed=5, restarts=4, lo=16, hi=96, rmin=2, rmax=8,
                     cmin=0.3, cmax=0.95, eta_h=0.01, build=True):
    """Problem list of the batched workload.

    ``default_rng(seed)`` draws, per problem b: three mode sizes ~ U{lo..hi}, a rank
    ~ U{rmin..rmax} and a collinearity ~ U[cmin, cmax].  Problem b's tensor uses seed
    5000 + b and its restarts use seeds 5000 + b + 1 + k.  With ``build=False`` only
    the descriptors are returned (no tensors).
    """
    rng = np.random.default_rng(seed)
    probs = []
    for b in range(count):
        dims = tuple(int(x) for x in rng.integers(lo, hi + 1, size=3))
        R = int(rng.integers(rmin, rmax + 1))
        c = float(rng.uniform(cmin, cmax))
        d = dict(b=b, dims=dims, R=R, c=c, eta_h=eta_h, tseed=5000 + b)
        if build:
            Z, _ = collinear_tensor(dims, R, c, eta_h, 0.0, 5000 + b)
            d["Z"] = Z
            d["starts"] = [uniform_start(dims, R, 5000 + b, k) for k in range(restarts)]
        probs.append(d)
    return probs


# ---------------------------------------------------------------------------
# Dense closed-form test problem of Section 6.3 (Table 4)
# ---------------------------------------------------------------------------
def dense_ijk(s):
    """The s x s x s tensor with entries (i^2 + j^2 + k^2)^(-1/2), i, j, k = 1..s
    (1-based), in Fortran order.  It is symmetric, so the layout of the modes
    does not matter."""
    i = np.arange(1, s + 1, dtype=np.float64)
    sq = i * i
    Z = 1.0 / np.sqrt(sq[:, None, None] + sq[None, :, None] + sq[None, None, :])
    return np.asfortranarray(Z)


# Table 4's problem parameters: test number -> (s, R).
DENSE_TESTS = {1: (50, 2), 2: (50, 3), 3: (50, 4), 4: (50, 5),
               5: (100, 2), 6: (100, 3), 7: (100, 4), 8: (100, 5),
               9: (200, 2), 10: (200, 3), 11: (200, 4), 12: (200, 5)}


def dense_case(s, R, run=0, n_t=2):
    """Inputs of one run of the dense problem, as a dict:

    - ``Z``: the tensor;
    - ``boot``: the boot factor matrices, also the start of standalone ALS;
    - ``tfms``: ``n_t`` test blocks;
    - ``coarsest``: the coarsening thresholds I_{n,coarsest} = 2R of every mode
      (with modes coarsened while larger than the threshold, this gives the level
      counts that Table 4 lists for all twelve tests);
    - ``seed``: the run's seed; the random coarsest-level start of the FMG cycle
      comes from ``dense_coarse_start(dims, R, seed)``.

    Every start is U(0,1) (the paper's initial guesses are standard uniform); the
    run's generator is ``default_rng(7000 + 100 s + 10 R + run)`` and draws the
    boot factors, then the test blocks in order."""
    Z = dense_ijk(s)
    seed = 7000 + 100 * s + 10 * R + run
    rng = np.random.default_rng(seed)
    dims = (s, s, s)
    boot = [np.ascontiguousarray(rng.random((s, R))) for _ in dims]
    tfms = [[np.ascontiguousarray(rng.random((s, R))) for _ in dims] for _ in range(n_t)]
    return dict(Z=Z, boot=boot, tfms=tfms, coarsest=[2 * R] * 3, seed=seed, s=s, R=R, run=run)


def dense_coarse_start(dims_coarse, R, seed):
    """U(0,1) start on the coarsest level for the FMG cycle (generator seed + 1)."""
    rng = np.random.default_rng(seed + 1)
    return [np.ascontiguousarray(rng.random((d, R))) for d in dims_coarse]


# ---------------------------------------------------------------------------
# Sparse test problem of Section 6.2 (Tables 2 and 3)
# ---------------------------------------------------------------------------
def laplacian_coo(d, s):
    """The finite-difference Laplacian on an s^d grid as an N = 2d mode tensor.

    The s^d x s^d matrix sum_k I_{s^(d-k)} (x) D (x) I_{s^(k-1)}, D = tridiag
    (-1, 2, -1) of size s, reshaped column-major to s x ... x s: modes 1..d are
    the digits of the row index and modes d+1..2d those of the column index
    (first digit fastest), so the entry at (i_1..i_d, j_1..j_d) is
    sum_k D(i_k, j_k) prod_{m != k} [i_m == j_m].  Returns (idx, vals, shape):
    0-based indices (nnz x N, int32) and values of the nonzero entries in
    increasing linear order (mode 1 fastest)."""
    rows = np.indices((s,) * d).reshape(d, -1, order="F").T   # row digits, first fastest
    idx_parts, val_parts = [], []
    idx_parts.append(np.concatenate([rows, rows], axis=1))
    val_parts.append(np.full(rows.shape[0], 2.0 * d))
    for k in range(d):
        for step in (-1, 1):
            ok = (rows[:, k] + step >= 0) & (rows[:, k] + step < s)
            r = rows[ok]
            c = r.copy()
            c[:, k] += step
            idx_parts.append(np.concatenate([r, c], axis=1))
            val_parts.append(np.full(r.shape[0], -1.0))
    idx = np.concatenate(idx_parts).astype(np.int64)
    vals = np.concatenate(val_parts)
    lin = np.zeros(idx.shape[0], dtype=np.int64)
    for m in range(2 * d - 1, -1, -1):
        lin = lin * s + idx[:, m]
    order = np.argsort(lin, kind="stable")
    return np.ascontiguousarray(idx[order].astype(np.int32)), np.ascontiguousarray(vals[order]), (s,) * (2 * d)


def coo_to_dense(idx, vals, shape):
    """Dense Fortran-order array holding the coordinate entries (zeros elsewhere)."""
    Z = np.zeros(shape, order="F")
    Z[tuple(np.asarray(idx, dtype=np.int64).T)] = vals
    return Z


# Table 2's problem parameters: test number -> (N, s, R).
LAPLACIAN_TESTS = {1: (4, 20, 4), 2: (4, 20, 5), 3: (4, 20, 6), 4: (4, 50, 2), 5: (4, 50, 3),
                   6: (4, 50, 4), 7: (6, 20, 2), 8: (6, 20, 3), 9: (6, 20, 4), 10: (8, 10, 2),
                   11: (8, 10, 3)}

# Coarsening thresholds I_{n,coarsest} by order: with modes coarsened while
# larger than the threshold they give the level counts Table 3 lists.
LAPLACIAN_COARSEST = {4: 10, 6: 5, 8: 3}


def laplacian_case(N, s, R, run=0, n_t=2):
    """Inputs of one run of the sparse problem, as a dict: ``idx``, ``vals``,
    ``shape`` (coordinate form), ``boot`` (boot factors, also the start of
    standalone ALS), ``tfms`` (n_t test blocks), ``coarsest`` and ``seed``.
    Starts are U(0,1) from ``default_rng(9000 + 1000 N + 10 s + R + 100000 run)``:
    boot factors first, then the test blocks in order."""
    idx, vals, shape = laplacian_coo(N // 2, s)
    seed = 9000 + 1000 * N + 10 * s + R + 100000 * run
    rng = np.random.default_rng(seed)
    boot = [np.ascontiguousarray(rng.random((s, R))) for _ in shape]
    tfms = [[np.ascontiguousarray(rng.random((s, R))) for _ in shape] for _ in range(n_t)]
    return dict(idx=idx, vals=vals, shape=shape, boot=boot, tfms=tfms,
                coarsest=[LAPLACIAN_COARSEST[N]] * N, seed=seed, N=N, s=s, R=R, run=run)

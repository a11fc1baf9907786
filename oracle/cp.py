"""CP model, gradient and ALS in plain FP64 NumPy (oracle; test infrastructure only).

Conventions.  A tensor is a NumPy array of logical shape (I_1, ..., I_N); modes
are numbered 0..N-1 here (1..N in the paper).  A factor list ``A`` holds N
matrices A^(n) of shape I_n x R whose columns are the mode-n factors (eq. (1)).

Readings of the paper taken here (each one is listed in the design notes):

* The update A <- Z_(n) Phi (Gamma)^dagger of Section 3 is evaluated with a
  Cholesky factorization of Gamma; if a pivot is <= R*eps*max(diag Gamma) (or the
  factorization fails) the Moore-Penrose pseudoinverse is used instead, built from
  a symmetric eigendecomposition with eigenvalues <= R*eps*lambda_max dropped.
* Normalization eq. (10) is applied after every complete sweep; a component with
  a zero-norm factor is left unchanged.  Sorting by decreasing lambda_r is stable
  and is applied by the drivers when a solve ends.
* The ten Gauss-Seidel iterations of Section 5.2 run over r = 1..R in increasing
  order with the newest values, warm-started from the current A^(n), row by row.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.linalg as sla

EPS = np.finfo(np.float64).eps


# ----------------------------------------------------------------------------
# Section 2: matricization, Khatri-Rao product, n-mode product
# ----------------------------------------------------------------------------
def unfold(Z, n):
    """Mode-n matricization Z_(n): mode-n fibers become the columns (Section 2).

    Column index of entry (i_1..i_N) is sum_{k != n} i_k J_k with
    J_k = prod_{m < k, m != n} I_m, i.e. lower modes vary fastest, which is the
    ordering under which eq. (5) holds.
    """
    Z = np.asarray(Z)
    return np.moveaxis(Z, n, 0).reshape(Z.shape[n], -1, order="F")


def fold(Mn, n, shape):
    """Inverse of :func:`unfold`."""
    shape = tuple(shape)
    rest = shape[:n] + shape[n + 1:]
    return np.moveaxis(Mn.reshape((shape[n],) + rest, order="F"), 0, n)


def khatri_rao(mats):
    """Column-wise Kronecker product mats[0] (.) mats[1] (.) ... (Section 2).

    Column r is a_r (x) b_r (x) ...; the row index of the last matrix varies
    fastest, as in the Kronecker product.
    """
    out = np.asarray(mats[0], dtype=np.float64)
    R = out.shape[1]
    for M in mats[1:]:
        out = (out[:, None, :] * np.asarray(M)[None, :, :]).reshape(-1, R)
    return out


def phi(A, n):
    """Phi^(n) = A^(N) (.) ... (.) A^(n+1) (.) A^(n-1) (.) ... (.) A^(1), eq. (7)."""
    N = len(A)
    return khatri_rao([A[m] for m in reversed(range(N)) if m != n])


def mode_product(Z, M, n):
    """n-mode product Z x_n M, defined through X_(n) = M Z_(n) (Section 2)."""
    shape = list(np.shape(Z))
    Xn = np.asarray(M) @ unfold(Z, n)
    shape[n] = M.shape[0]
    return fold(Xn, n, shape)


# ----------------------------------------------------------------------------
# CP model, Gram matrices, MTTKRP, objective and gradient (Sections 1, 3, 6)
# ----------------------------------------------------------------------------
def grams(A):
    """Upsilon^(n) = A^(n)^T A^(n) for every mode (text after eq. (8))."""
    return [a.T @ a for a in A]


def gamma(G, n):
    """Gamma^(n): Hadamard product of all Upsilon^(m), m != n, eq. (8)."""
    R = G[0].shape[0]
    out = np.ones((R, R))
    for m, g in enumerate(G):
        if m != n:
            out = out * g
    return out


def mttkrp(Z, A, n):
    """Z_(n) Phi^(n) with an explicit Khatri-Rao matrix (the product in eq. (6))."""
    return unfold(Z, n) @ phi(A, n)


def mttkrp_coo(idx, vals, shape, A, n):
    """Z_(n) Phi^(n) of a tensor given by its nonzero entries (Section 6.2):
    M(i_n, r) = sum over the stored entries z_{i_1..i_N} of
    z prod_{m != n} A^(m)(i_m, r); every other entry is zero and adds nothing.
    ``idx``: nnz x N 0-based indices (no index stored twice), ``vals``: nnz."""
    idx = np.asarray(idx, dtype=np.int64)
    R = A[0].shape[1]
    W = np.asarray(vals, dtype=np.float64)[:, None] * np.ones((1, R))
    for m in range(len(shape)):
        if m != n:
            W = W * A[m][idx[:, m], :]
    M = np.zeros((shape[n], R))
    np.add.at(M, idx[:, n], W)
    return M


def full(A):
    """[[A^(1), ..., A^(N)]] = sum_r a_r^(1) o ... o a_r^(N), eq. (1)."""
    R = A[0].shape[1]
    out = None
    for r in range(R):
        t = functools.reduce(np.multiply.outer, [a[:, r] for a in A])
        out = t if out is None else out + t
    return out


def objective(Z, A):
    """f = 1/2 ||Z - [[A]]||^2 from the formed residual, eq. (2)."""
    D = np.asarray(Z) - full(A)
    return 0.5 * float(np.sum(D * D))


def objective_fused(norm2Z, A_last, M_last, G):
    """Same f from quantities a sweep already has, for the last mode n = N:

    ||[[A]]||^2 = 1^T (*_n Upsilon^(n)) 1 and <Z, [[A]]> = <A^(N), Z_(N) Phi^(N)>.
    """
    H = np.ones_like(G[0])
    for g in G:
        H = H * g
    return 0.5 * (norm2Z - 2.0 * float(np.sum(A_last * M_last)) + float(np.sum(H)))


def gradient(Z, A):
    """G^(n) = -Z_(n) Phi^(n) + A^(n) Gamma^(n) for every mode, eq. (6)."""
    G = grams(A)
    return [-mttkrp(Z, A, n) + A[n] @ gamma(G, n) for n in range(len(A))]


def grad_norm(Z, A):
    """g = (sum_n ||G^(n)||^2)^(1/2) / ||Z||, eq. (30)."""
    Gs = gradient(Z, A)
    s = sum(float(np.sum(g * g)) for g in Gs)
    return np.sqrt(s) / np.linalg.norm(np.asarray(Z).ravel())


def fit(Z, A):
    """1 - ||Z - [[A]]|| / ||Z|| (the paper uses f and g; this is the derived fit)."""
    nz = np.linalg.norm(np.asarray(Z).ravel())
    return 1.0 - np.sqrt(2.0 * objective(Z, A)) / nz


# ----------------------------------------------------------------------------
# R x R solves
# ----------------------------------------------------------------------------
def solve_gamma(B, Gam, return_info=False):
    """X with X Gamma = B, i.e. X = B Gamma^dagger (Section 3, ALS update).

    Cholesky first; pseudoinverse fallback when a pivot is <= R*eps*max(diag).
    """
    R = Gam.shape[0]
    dmax = float(np.max(np.diag(Gam))) if R else 0.0
    thr = R * EPS * dmax
    fallback = False
    try:
        L = np.linalg.cholesky(Gam)
        if np.min(np.diag(L)) ** 2 <= thr or dmax <= 0:
            fallback = True
    except np.linalg.LinAlgError:
        fallback = True
    if not fallback:
        Y = sla.solve_triangular(L, B.T, lower=True)
        X = sla.solve_triangular(L.T, Y, lower=False).T
    else:
        w, V = np.linalg.eigh(Gam)
        lmax = float(np.max(w)) if R else 0.0
        keep = w > R * EPS * lmax
        inv = np.zeros_like(w)
        inv[keep] = 1.0 / w[keep]
        X = B @ (V * inv) @ V.T
    return (X, fallback) if return_info else X


def gauss_seidel(X0, Gam, B, iters):
    """``iters`` Gauss-Seidel iterations on X Gamma = B, one system per row (Sec. 5.2).

    Each row x solves Gamma x^T = b^T (Gamma is symmetric).  Components are
    visited r = 1..R with the newest values; a zero diagonal leaves x_r as is.
    Rows are independent, so they are updated together.
    """
    X = np.array(X0, dtype=np.float64, copy=True)
    R = Gam.shape[0]
    for _ in range(iters):
        for r in range(R):
            d = Gam[r, r]
            if d == 0.0:
                continue
            s = B[:, r] - X @ Gam[:, r] + X[:, r] * d
            X[:, r] = s / d
    return X


# ----------------------------------------------------------------------------
# Normalization and ordering (eq. (10) and the remark after it)
# ----------------------------------------------------------------------------
def component_norms(A):
    return np.array([np.linalg.norm(a, axis=0) for a in A])   # N x R


def normalize(A):
    """a_r^(n) -> lambda_r a_r^(n)/||a_r^(n)||, lambda_r = (prod_n ||a_r^(n)||)^(1/N)."""
    N = len(A)
    nr = component_norms(A)
    ok = np.all(nr > 0, axis=0)
    lam = np.ones(nr.shape[1])
    lam[ok] = np.prod(nr[:, ok], axis=0) ** (1.0 / N)
    out = []
    for n in range(N):
        s = np.ones(nr.shape[1])
        s[ok] = lam[ok] / nr[n, ok]
        out.append(A[n] * s)
    return out


def weights(A):
    """lambda_r of eq. (10) for the current factors."""
    nr = component_norms(A)
    return np.prod(nr, axis=0) ** (1.0 / len(A))


def sort_components(A):
    """Order the rank-one terms by decreasing lambda_r (stable)."""
    lam = weights(A)
    order = np.argsort(-lam, kind="stable")
    return [a[:, order] for a in A], order


# ----------------------------------------------------------------------------
# ALS / block nonlinear Gauss-Seidel (Section 3; with a right-hand side, Sec. 5.2)
# ----------------------------------------------------------------------------
def als_sweep(Z, A, F=None, solver="chol", gs_iters=10, normalize_after=True,
              info=None):
    """One BNGS iteration on A^(n) Gamma^(n) = Z_(n) Phi^(n) + F^(n), n = 1..N.

    ``solver='chol'`` is the ALS update with Gamma^dagger (Section 3);
    ``solver='gs'`` runs ``gs_iters`` Gauss-Seidel iterations (eq. (29)).
    ``info`` (dict, optional) collects 'fallbacks' and the last mode's MTTKRP.
    """
    A = [np.array(a, dtype=np.float64, copy=True) for a in A]
    N = len(A)
    for n in range(N):
        G = grams(A)
        Gam = gamma(G, n)
        M = mttkrp(Z, A, n)
        rhs = M if F is None else M + F[n]
        if solver == "chol":
            A[n], fb = solve_gamma(rhs, Gam, return_info=True)
            if info is not None:
                info["fallbacks"] = info.get("fallbacks", 0) + int(fb)
        elif solver == "gs":
            A[n] = gauss_seidel(A[n], Gam, rhs, gs_iters)
        else:
            raise ValueError(solver)
        if info is not None and n == N - 1:
            info["M_last"] = M
            info["inner_last"] = float(np.sum(A[n] * M))
            info["grams"] = grams(A)
    if normalize_after:
        A = normalize(A)
    return A


def als(Z, A0, max_sweeps=10000, fit_tol=1e-12, g_tol=None, record="fused",
        solver="chol", sort_at_end=True):
    """Standalone ALS driver (Section 3, caps of Section 6).

    Stops when |fit_k - fit_{k-1}| <= fit_tol * fit_k, when g < g_tol (if given),
    or after ``max_sweeps`` sweeps.  ``record='fused'`` evaluates f per sweep with
    :func:`objective_fused` (cheap), ``'direct'`` with :func:`objective`.
    Returns (A, history dict).
    """
    A = [np.array(a, dtype=np.float64) for a in A0]
    nz2 = float(np.sum(np.asarray(Z) ** 2))
    hist = {"fit": [], "f": [], "g": []}
    prev = None
    k = 0
    for k in range(1, max_sweeps + 1):
        info = {}
        A = als_sweep(Z, A, solver=solver, info=info)
        if record == "direct":
            fk_obj = objective(Z, A)
        else:
            # <A^(N), M^(N)> and the Grams are taken before normalization;
            # normalization leaves [[A]] (hence f) unchanged
            H = np.ones_like(info["grams"][0])
            for g in info["grams"]:
                H = H * g
            fk_obj = 0.5 * (nz2 - 2.0 * info["inner_last"] + float(np.sum(H)))
        fk = 1.0 - np.sqrt(max(2.0 * fk_obj, 0.0) / nz2)
        hist["f"].append(fk_obj)
        hist["fit"].append(fk)
        if g_tol is not None:
            gk = grad_norm(Z, A)
            hist["g"].append(gk)
            if gk < g_tol:
                break
        if fit_tol and prev is not None and abs(fk - prev) <= fit_tol * abs(fk):
            break
        prev = fk
    hist["sweeps"] = k
    if sort_at_end:
        A, _ = sort_components(A)
    return A, hist

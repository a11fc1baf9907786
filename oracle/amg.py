"""Multilevel parts of the method in plain FP64 NumPy (oracle; test infrastructure only).

Section 4 (multiplicative setup), Section 5 (FAS solve) and the Section 6.1
driver rules.  Mode indices are 0-based; point indices are 0-based, so the
paper's odd (1-based) coarse points are the even 0-based indices here.

Readings of the paper taken here (each one is listed in the design notes):

* Coarse size I_c = ceil(I/2); the last point of an even-length mode is a fine
  point with the single coarse neighbour alpha(i-1) (Sec. 4.3 "except possibly at
  the right endpoint").
* Coarse Gram of Sec. 4.1 is read as A_c^T B A_c (the printed formula mixes
  A_c and A, which is dimensionally impossible).
* Least-squares weights eq. (20) use the gradient of each block at its current
  iterate (after the nu_1 relaxations); ||G^(n)|| is floored at
  1e-8 ||Z_(n) Phi^(n)|| (the mode an ALS sweep solved last has a gradient that
  vanishes identically, so its computed value is rounding noise).
* Coarse right-hand side for modes that are not coarsened: Algorithm 2 writes
  F_c = F, which loses the FAS fixed point unless A lies in range(P) for every
  other mode; the default here is the tau-corrected form
  F_c = F - H(A) + H_c(A~_c) ('tau'); the printed form is available ('literal').
  Both coincide whenever every mode is coarsened.
* Normalization is applied after each BNGS iteration only on the top level of a
  cycle (where F = 0); the setup phase normalizes on every level (it solves a
  plain CP problem there).
* FMG (Alg. 3): the number of coarsest-level ALS iterations nu is not fixed by
  the paper; the default is the setup phase's nu_c = 100.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import cp

# Table 1 parameters
SETUP_PARAMS = dict(nu1=5, nu2=5, nuc=100, nt=2)
SETUP_PARAMS_NO_NT = dict(nu1=5, nu2=5, nuc=100)   # keyword form for setup_phase
FAS_PARAMS = dict(nu1=1, nu2=1, nuc=50, gs_iters=10)


# ----------------------------------------------------------------------------
# Section 4.3: geometric coarsening and the sparsity of P
# ----------------------------------------------------------------------------
def coarse_size(I):
    return (I + 1) // 2


def interp_sets(I):
    """Coarse points C (0-based even), fine points F and C_i for each fine i."""
    C = list(range(0, I, 2))
    F = list(range(1, I, 2))
    Ci = {}
    for i in F:
        Ci[i] = [(i - 1) // 2] + ([(i + 1) // 2] if i + 1 < I else [])
    return C, F, Ci


def interp_from_weights(I, w):
    """Dense P (I x I_c) from per-row weights w (I x 2): 1 on coarse rows."""
    Ic = coarse_size(I)
    P = np.zeros((I, Ic))
    C, F, Ci = interp_sets(I)
    for i in C:
        P[i, i // 2] = 1.0
    for i in F:
        for k, j in enumerate(Ci[i]):
            P[i, j] = w[i, k]
    return P


# ----------------------------------------------------------------------------
# Section 4.4: least-squares interpolation weights
# ----------------------------------------------------------------------------
def ls_interp_weights(U, wts):
    """Weights w_ij from the weighted LS fits eq. (19) by normal equations.

    U is I x n_f (columns are the vectors to fit); wts (n_f) the fit weights.
    Coarse values are injections: (u_{k,c})_j = u_k at fine point 2j.
    Returns w (I x 2); coarse rows are zero.
    """
    I, nf = U.shape
    _, F, Ci = interp_sets(I)
    W = np.asarray(wts, dtype=np.float64)
    w = np.zeros((I, 2))
    for i in F:
        X = np.stack([U[2 * j, :] for j in Ci[i]], axis=1)   # nf x |C_i|
        y = U[i, :]
        XtW = X.T * W
        w[i, : X.shape[1]] = np.linalg.solve(XtW @ X, XtW @ y)
    return w


# ||G^(n)|| below this fraction of ||Z_(n) Phi^(n)|| is taken at that level
GRAD_FLOOR = 1e-8


def block_weight(Z, A, n):
    """w_r = ||A^(n)||^2 / ||G^(n)||^2 for one block of factor matrices, eq. (20),
    G^(n) = A^(n) Gamma^(n) - Z_(n) Phi^(n) (eq. (6)).

    After an ALS sweep the gradient of the mode solved last vanishes identically
    (the update solves G^(n) = 0 and the rescaling of eq. (10) keeps it zero), so
    its computed norm is rounding noise and the ratio would be arbitrary.  The
    norm is therefore floored at GRAD_FLOOR * ||Z_(n) Phi^(n)||, far below any
    gradient the setup phase acts on and far above rounding.
    """
    M = cp.mttkrp(Z, A, n)
    G = A[n] @ cp.gamma(cp.grams(A), n) - M
    gn2 = max(float(np.sum(G * G)), GRAD_FLOOR * GRAD_FLOOR * float(np.sum(M * M)))
    return float(np.sum(A[n] * A[n])) / gn2


def build_interp(Z, tfms, bfm, n, use_bfm):
    """Weights of P^(n) fitted to the TFMs of every test block (+ the BFMs)."""
    cols, wts = [], []
    blocks = list(tfms) + ([bfm] if use_bfm else [])
    for blk in blocks:
        cols.append(blk[n])
        wts.extend([block_weight(Z, blk, n)] * blk[n].shape[1])
    U = np.concatenate(cols, axis=1)
    return ls_interp_weights(U, np.array(wts))


# ----------------------------------------------------------------------------
# Section 4.1: B = P^T P, Cholesky, P^ = P L^{-T}, R^ = P^^T, coarse tensor
# ----------------------------------------------------------------------------
def transfer(P):
    """Return (B, L, Phat) with B = P^T P = L L^T and Phat = P L^{-T} (Alg. 1 steps 4-6)."""
    B = P.T @ P
    L = np.linalg.cholesky(B)
    Phat = sla.solve_triangular(L, P.T, lower=True).T
    return B, L, Phat


def restrict_tensor(Z, Rhat):
    """Z x_{n in I_c} R^^(n), eq. (15); ``Rhat[n] is None`` means the identity."""
    out = np.asarray(Z, dtype=np.float64)
    for n, Rn in enumerate(Rhat):
        if Rn is not None:
            out = cp.mode_product(out, Rn, n)
    return out


def restrict_factors(Phat, A):
    """A~_c^(n) = R^^(n) A^(n) for coarsened modes, A^(n) otherwise, eq. (21)."""
    return [A[n].copy() if Phat[n] is None else Phat[n].T @ A[n] for n in range(len(A))]


def prolong(Phat, Ac):
    """A_CGC^(n) = P^^(n) A^_c^(n) for coarsened modes, A^_c^(n) otherwise, eq. (22)."""
    return [Ac[n].copy() if Phat[n] is None else Phat[n] @ Ac[n] for n in range(len(Ac))]


def fas_correct(Phat, A, Ac, At):
    """A^(n) + P^^(n)(A_c^(n) - A~_c^(n)) (identity for modes not coarsened), eq. (28)."""
    out = []
    for n in range(len(A)):
        d = Ac[n] - At[n]
        out.append(A[n] + (d if Phat[n] is None else Phat[n] @ d))
    return out


# ----------------------------------------------------------------------------
# Level hierarchy
# ----------------------------------------------------------------------------
@dataclass
class Level:
    Z: np.ndarray
    Phat: list = field(default_factory=list)   # per mode: I_n x I_n,c (to next level) or None
    weights: list = field(default_factory=list)   # per mode: the I_n x 2 weights P^ was built from

    @property
    def dims(self):
        return self.Z.shape


def hierarchy_from_weights(Z, weights_per_level, coarsest):
    """Build levels from given interpolation weights (list per level of per-mode w or None)."""
    levels = []
    cur = np.asarray(Z, dtype=np.float64)
    for wl in weights_per_level:
        Ph, Ws = [], []
        for n, In in enumerate(cur.shape):
            if In > coarsest[n] and wl[n] is not None:
                Ph.append(transfer(interp_from_weights(In, wl[n]))[2])
                Ws.append(np.asarray(wl[n]))
            else:
                Ph.append(None)
                Ws.append(None)
        if all(p is None for p in Ph):
            break
        levels.append(Level(cur, Ph, Ws))
        cur = restrict_tensor(cur, [None if p is None else p.T for p in Ph])
    levels.append(Level(cur, [None] * cur.ndim))
    return levels


# ----------------------------------------------------------------------------
# Section 5: FAS operators, relaxation and the CP-FAS V-cycle (Algorithm 2)
# ----------------------------------------------------------------------------
def fas_H(Z, A):
    """H^(n)(A) = A^(n) Gamma^(n) - Z_(n) Phi^(n) for every mode, eq. (23)."""
    G = cp.grams(A)
    return [A[n] @ cp.gamma(G, n) - cp.mttkrp(Z, A, n) for n in range(len(A))]


def bngs(Z, A, F, gs_iters=10, normalize_after=False):
    """One BNGS iteration on H(A) = F with Gauss-Seidel inner solves, eq. (29)."""
    return cp.als_sweep(Z, A, F=F, solver="gs", gs_iters=gs_iters,
                        normalize_after=normalize_after)


def fas_vcycle(levels, F, A, l=0, top=0, nu1=1, nu2=1, nuc=50, gs_iters=10,
               ic_rule="tau"):
    """Algorithm 2 (CP-FAS V-cycle) on level ``l``; normalization only on level ``top``."""
    lev = levels[l]
    norm = (l == top)
    if l == len(levels) - 1:
        for _ in range(nuc):
            A = bngs(lev.Z, A, F, gs_iters, norm)
        return A
    for _ in range(nu1):
        A = bngs(lev.Z, A, F, gs_iters, norm)
    Ph = lev.Phat
    At = restrict_factors(Ph, A)
    H = fas_H(lev.Z, A)
    Hc = fas_H(levels[l + 1].Z, At)
    Fc = []
    for n in range(len(A)):
        if Ph[n] is not None:
            Fc.append(Hc[n] + Ph[n].T @ (F[n] - H[n]))
        elif ic_rule == "literal":
            Fc.append(F[n].copy())
        else:
            Fc.append(F[n] - H[n] + Hc[n])
    Ac = fas_vcycle(levels, Fc, At, l + 1, top, nu1, nu2, nuc, gs_iters, ic_rule)
    A = fas_correct(Ph, A, Ac, At)
    for _ in range(nu2):
        A = bngs(lev.Z, A, F, gs_iters, norm)
    return A


def zeros_like_factors(A):
    return [np.zeros_like(a) for a in A]


def fmg_cycle(levels, A_coarse_init, nu=100, **fas):
    """Algorithm 3 (FMG-CP-FAS): nu ALS iterations on the coarsest level, then
    interpolate and run one CP-FAS V-cycle with F = 0 on each finer level."""
    L = len(levels)
    A = [np.array(a, dtype=np.float64) for a in A_coarse_init]
    for _ in range(nu):
        A = cp.als_sweep(levels[L - 1].Z, A)
    for l in range(L - 1, 0, -1):
        A = prolong(levels[l - 1].Phat, A)
        A = fas_vcycle(levels, zeros_like_factors(A), A, l=l - 1, top=l - 1, **fas)
    return A


# ----------------------------------------------------------------------------
# Section 4.2 / Algorithm 1: CP-AMG-mult setup V-cycle and down-sweep
# ----------------------------------------------------------------------------
def mult_vcycle(Z, A, tfms, coarsest, first_cycle, nu1=5, nu2=5, nuc=100,
                levels_out=None):
    """Algorithm 1.  Returns (updated BFMs, updated fine TFMs, levels list)."""
    if levels_out is None:
        levels_out = []
    Z = np.asarray(Z, dtype=np.float64)
    N = Z.ndim
    Ic = [n for n in range(N) if Z.shape[n] > coarsest[n]]
    if not Ic:
        for _ in range(nuc):
            A = cp.als_sweep(Z, A)
        levels_out.append(Level(Z, [None] * N))
        return A, tfms, levels_out
    for _ in range(nu1):
        tfms = [cp.als_sweep(Z, T) for T in tfms]
        A = cp.als_sweep(Z, A)
    Ph = [None] * N
    Ws = [None] * N
    for n in Ic:
        w = build_interp(Z, tfms, A, n, use_bfm=not first_cycle)
        Ws[n] = w
        Ph[n] = transfer(interp_from_weights(Z.shape[n], w))[2]
    At = restrict_factors(Ph, A)
    tfms_c = [restrict_factors(Ph, T) for T in tfms]
    Zc = restrict_tensor(Z, [None if p is None else p.T for p in Ph])
    levels_out.append(Level(Z, Ph, Ws))
    Ac, _, _ = mult_vcycle(Zc, At, tfms_c, coarsest, first_cycle, nu1, nu2, nuc, levels_out)
    A = prolong(Ph, Ac)
    for _ in range(nu2):
        A = cp.als_sweep(Z, A)
    return A, tfms, levels_out


def down_sweep(Z, A_boot, tfms, coarsest, nu1=5, use_bfm=True):
    """Downward half of Algorithm 1 that rebuilds the transfer operators.

    TFMs are relaxed; the boot factors are only restricted (not updated), as the
    rebuild of Section 6.1 prescribes.  Returns (levels, updated fine TFMs).
    """
    levels = []
    Z = np.asarray(Z, dtype=np.float64)
    B = [np.array(a) for a in A_boot]
    fine_tfms = None
    while True:
        N = Z.ndim
        Ic = [n for n in range(N) if Z.shape[n] > coarsest[n]]
        if not Ic:
            levels.append(Level(Z, [None] * N))
            break
        for _ in range(nu1):
            tfms = [cp.als_sweep(Z, T) for T in tfms]
        if fine_tfms is None:
            fine_tfms = tfms
        Ph = [None] * N
        Ws = [None] * N
        for n in Ic:
            w = build_interp(Z, tfms, B, n, use_bfm=use_bfm)
            Ws[n] = w
            Ph[n] = transfer(interp_from_weights(Z.shape[n], w))[2]
        levels.append(Level(Z, Ph, Ws))
        B = restrict_factors(Ph, B)
        tfms = [restrict_factors(Ph, T) for T in tfms]
        Z = restrict_tensor(Z, [None if p is None else p.T for p in Ph])
    return levels, (fine_tfms if fine_tfms is not None else tfms)


def setup_phase(Z, A0, tfms0, coarsest, max_cycles=5, check_after=3, eps=0.1,
                **mult):
    """Setup cycles of Section 6.1: stop when g_new > (1 - eps) g_old (eq. (32)),
    checked once ``check_after`` cycles have completed, at most ``max_cycles``."""
    A, tfms = A0, tfms0
    g_old = cp.grad_norm(Z, A)
    levels = None
    hist = []
    for c in range(max_cycles):
        A, tfms, levels = mult_vcycle(Z, A, tfms, coarsest, first_cycle=(c == 0), **mult)
        g_new = cp.grad_norm(Z, A)
        hist.append(g_new)
        if c + 1 >= check_after and g_new > (1.0 - eps) * g_old:
            break
        g_old = g_new
    return A, tfms, levels, hist


def solve_phase(Z, A, levels, tfms, coarsest, tau=1e-10, max_cycles=500,
                stagnation_after=5, nu1_setup=5, info=None, **fas):
    """FAS cycles until g < tau with one stagnation-triggered rebuild (Section 6.1).
    If ``info`` is a dict, info["rebuilt"] tells whether the rebuild happened."""
    g_old = cp.grad_norm(Z, A)
    rebuilt = False
    hist = []
    for c in range(max_cycles):
        A_new = fas_vcycle(levels, zeros_like_factors(A), A, **fas)
        g_new = cp.grad_norm(Z, A_new)
        if c + 1 > stagnation_after and g_new >= g_old and not rebuilt:
            levels, tfms = down_sweep(Z, A, tfms, coarsest, nu1=nu1_setup)
            rebuilt = True
            continue
        A, g_old = A_new, g_new
        hist.append(g_new)
        if g_new < tau:
            break
    if info is not None:
        info["rebuilt"] = rebuilt
    return A, levels, hist


def multilevel(Z, A0, tfms0, coarsest, tau=1e-10, max_cycles=500, setup=None, fas=None):
    """'Multilevel' of Section 6.1 (no FMG): setup cycles stopped by eq. (32),
    then solve cycles from the setup's boot factors on the setup's levels until
    g < tau, with the one stagnation rebuild.  Returns (A, info) with the fields
    of ``multilevel_fmg`` except 'fmg'."""
    setup = dict(setup or {})
    fas = dict(fas or {})
    A, tfms, levels, shist = setup_phase(Z, A0, tfms0, coarsest, **setup)
    out = {}
    A, levels, hist = solve_phase(Z, A, levels, tfms, coarsest, tau, max_cycles,
                                  nu1_setup=setup.get("nu1", 5), info=out, **fas)
    info = dict(setup=shist, solve=hist, rebuilt=out["rebuilt"], levels=len(levels),
                iterations=len(shist) + len(hist))
    return A, info


def multilevel_fmg(Z, A0, tfms0, coarsest, coarse_start, tau=1e-10, max_cycles=500,
                   fmg_nu=100, setup=None, fas=None):
    """'Multilevel + FMG' of Section 6.1.

    1. Setup cycles (Algorithm 1) from the boot factors A0 and test blocks tfms0,
       stopped by eq. (32) as in ``setup_phase``.
    2. One FMG-CP-FAS cycle (Algorithm 3) over the setup's levels, started from
       ``coarse_start`` on the coarsest level: its result is the new
       approximation to the boot factors.
    3. The transfer operators are rebuilt by one down-sweep of Algorithm 1 with
       these boot factors (the test blocks are relaxed, the boot factors are not).
    4. Solve cycles (``solve_phase``) from the FMG result until g < tau.

    Returns (A, info) with info = dict(setup=g after each setup cycle,
    fmg=g after the FMG cycle, solve=g after each kept solve cycle,
    rebuilt=whether the solve phase rebuilt its operators, levels=level count,
    iterations=setup cycles + solve cycles)."""
    setup = dict(setup or {})
    fas = dict(fas or {})
    A, tfms, levels, shist = setup_phase(Z, A0, tfms0, coarsest, **setup)
    A = fmg_cycle(levels, coarse_start, nu=fmg_nu, **fas)
    g_fmg = cp.grad_norm(Z, A)
    nu1 = setup.get("nu1", 5)
    levels, tfms = down_sweep(Z, A, tfms, coarsest, nu1=nu1)
    out = {}
    A, levels, hist = solve_phase(Z, A, levels, tfms, coarsest, tau, max_cycles,
                                  nu1_setup=nu1, info=out, **fas)
    rebuilt = out["rebuilt"]
    info = dict(setup=shist, fmg=g_fmg, solve=hist, rebuilt=rebuilt, levels=len(levels),
                iterations=len(shist) + len(hist))
    return A, info


def default_coarsest(dims, R, target=None):
    """I_n,coarsest: ``target`` if given, else max(R, 2) (Sec. 4.5 suggests >= R)."""
    return [target if target is not None else max(R, 2) for _ in dims]


def n_levels(dims, coarsest):
    L = 1
    d = list(dims)
    while any(d[n] > coarsest[n] for n in range(len(d))):
        d = [coarse_size(x) if x > coarsest[n] else x for n, x in enumerate(d)]
        L += 1
    return L


__all__ = [name for name in dir() if not name.startswith("_") and name not in ("math",)]

"""Host-side solve loops on top of the C ABI (stopping decisions only).

Each loop enqueues a chunk of device work, reads back a few scalars and decides
whether to continue; all arithmetic happens in libcpamg's kernels.

Stopping rules (Section 6 of the paper uses the gradient measure g < 1e-10 with
caps of 1e4 ALS iterations and 500 multilevel iterations; the workloads here
stop on the relative fit change):
  * ALS / FP64 phase: |fit_k - fit_{k-1}| <= fit_tol * fit_k, fit = 1 - ||Z-[[A]]||/||Z||
  * mixed form: FP32 sweeps until the mean per-sweep fit gain over a chunk of
    sweeps is <= tol32 * fit, then FP64 sweeps as above.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import api
from ._lib import CP_FP64, CP_MIXED, CP_SOLVE_CHOL, CP_SOLVE_GS


def _torch():
    import torch
    return torch


@dataclass
class SolveResult:
    sweeps: int = 0
    sweeps32: int = 0
    sweeps64: int = 0
    fits: list = field(default_factory=list)
    final_fit: float = float("nan")
    converged: bool = False


def fit_from_f(f, norm2):
    return 1.0 - math.sqrt(max(2.0 * f, 0.0) / norm2)


def _copy_factors(dst, src):
    for d, s in zip(dst.mats, src.mats):
        d.copy_(s)
    if dst.mats32 is not None and src.mats32 is not None:
        for d, s in zip(dst.mats32, src.mats32):
            d.copy_(s)


def als_solve(ctx, Z, A, max_sweeps=10000, fit_tol=1e-12, chunk=16, prec=CP_FP64,
              solver=CP_SOLVE_CHOL, sort_at_end=True, exact_stop=True):
    """Standalone ALS (Section 3) with the fused objective read back per chunk.

    The device runs ``chunk`` sweeps between two reads of the fit history.
    With ``exact_stop`` the factors are kept as they were before each chunk, and
    when the stopping rule holds after sweep j < chunk of a chunk they are put
    back and exactly j sweeps are run again (the kernels are deterministic, so
    this reproduces the first j sweeps): the solve ends on the sweep where the
    rule first holds.  Without it the rest of the chunk runs too.
    """
    torch = _torch()
    norm2 = float(Z.norm2.item())
    fh = torch.zeros(chunk, dtype=torch.float64, device=Z.device)
    res = SolveResult()
    prev = None
    snap = A.clone() if (exact_stop and fit_tol) else None
    while res.sweeps < max_sweeps:
        k = min(chunk, max_sweeps - res.sweeps)
        if snap is not None:
            _copy_factors(snap, A)
        api.cp_als_sweep(ctx, Z, A, None, k, solver, 10, True, prec, fh)
        fv = fh[:k].cpu().numpy()
        stop_at = None
        for j in range(k):
            fit = fit_from_f(float(fv[j]), norm2)
            if fit_tol and prev is not None and abs(fit - prev) <= fit_tol * abs(fit):
                stop_at = j + 1
                break
            prev = fit
        if stop_at is None:
            res.fits.extend(fit_from_f(float(x), norm2) for x in fv)
            res.sweeps += k
            continue
        res.converged = True
        if snap is not None and stop_at < k:
            _copy_factors(A, snap)
            api.cp_als_sweep(ctx, Z, A, None, stop_at, solver, 10, True, prec, fh)
            fv = fh[:stop_at].cpu().numpy()
            res.fits.extend(fit_from_f(float(x), norm2) for x in fv)
            res.sweeps += stop_at
        else:
            res.fits.extend(fit_from_f(float(x), norm2) for x in fv)
            res.sweeps += k
        break
    if sort_at_end:
        api.cp_sort(ctx, A)
    res.final_fit = res.fits[-1] if res.fits else float("nan")
    return res


def exact_fit(ctx, Z, A, f=None, norm2=None):
    """Fit 1 - ||Z - [[A]]|| / ||Z|| from the exact objective.  In a loop, pass
    ``f`` (a device scalar to reuse) and ``norm2`` (||Z||^2 read once) to spare
    the allocation and the second read-back per call."""
    torch = _torch()
    if f is None:
        f = torch.zeros(1, dtype=torch.float64, device=Z.device)
    else:
        f.zero_()
    api.cp_objective(ctx, Z, A, exact=True, f=f)
    if norm2 is None:
        norm2 = float(Z.norm2.item())
    return fit_from_f(float(f.item()), norm2)


def mixed_solve(ctx, Z, A, tol32=1e-9, tol64=1e-12, chunk32=16, max_sweeps=10000, chunk64=16,
                tol32_fp64=1e-11):
    """Mixed form: FP32-contraction sweeps, then FP64 refinement sweeps.

    The FP32 phase runs in chunks of ``chunk32`` sweeps.  Its own fused
    objective (from the FP32 contraction) raises the alarm when the mean
    per-sweep gain over a chunk is <= tol32 * fit; a negative gain means the
    FP32 values have reached their noise floor.  That noise is larger than the
    late gains, so the alarm comes hundreds of sweeps before the FP32 sweeps
    stop tracking the FP64 trajectory.  With ``tol32_fp64`` (and an FP64 copy
    of Z) the alarm is therefore checked: from then on the fit after each chunk
    comes from the objective with an FP64 contraction (cp_objective's fused
    identity, one FP64 MTTKRP), and the phase ends when that per-sweep gain is
    <= tol32_fp64 * fit.  Without it the alarm ends the phase.

    The FP64 phase then runs until the per-sweep fit change is <= tol64 * fit.
    """
    torch = _torch()
    norm2 = float(Z.norm2.item())
    fh = torch.zeros(chunk32, dtype=torch.float64, device=Z.device)
    check = bool(tol32_fp64) and Z.z64 is not None
    fbuf = torch.zeros(1, dtype=torch.float64, device=Z.device)

    def fit_fp64():
        fbuf.zero_()
        api.cp_objective(ctx, Z, A, exact=False, f=fbuf, prec=CP_FP64)
        return fit_from_f(float(fbuf.item()), norm2)

    prev = None   # FP64-contraction fit after the last chunk, once the alarm came
    res = SolveResult()
    while res.sweeps < max_sweeps:
        k = min(chunk32, max_sweeps - res.sweeps)
        api.cp_als_sweep(ctx, Z, A, None, k, CP_SOLVE_CHOL, 10, True, CP_MIXED, fh)
        fits = [fit_from_f(float(x), norm2) for x in fh[:k].cpu().numpy()]
        res.fits.extend(fits)
        res.sweeps += k
        res.sweeps32 += k
        if prev is not None:
            cur = fit_fp64()
            gain, prev = (cur - prev) / k, cur
            if gain <= tol32_fp64 * abs(cur):
                break
        elif k >= 2 and (fits[-1] - fits[0]) / (k - 1) <= tol32 * abs(fits[-1]):
            if not check:
                break
            prev = fit_fp64()
    r64 = als_solve(ctx, Z, A, max_sweeps=max(1, max_sweeps - res.sweeps), fit_tol=tol64,
                    chunk=chunk64, prec=CP_FP64)
    res.sweeps64 = r64.sweeps
    res.sweeps += r64.sweeps
    res.fits.extend(r64.fits)
    res.final_fit = r64.final_fit
    res.converged = r64.converged
    return res


def build_hierarchy(ctx, Z, weights, prec=CP_FP64, fp32=False, fp64=True):
    """Levels for cp_fas_vcycle from interpolation weights.

    ``weights[l][n]``: (I_n x 2) numpy weights of mode n on level l, or None when
    that mode is not coarsened.  Operator prep (B, L, P^) and the coarse tensors
    run on the device (cp_transfer_build, cp_restrict).  Coarse tensors are kept
    in FP64 (``fp64``) and/or FP32 (``fp32``, implied by the mixed form).
    """
    torch = _torch()
    levels = []
    cur = Z
    for wl in weights:
        ph, wd = [], []
        for n, d in enumerate(cur.dims):
            if wl[n] is None:
                ph.append(None)
                wd.append(None)
                continue
            w = torch.from_numpy(np.ascontiguousarray(wl[n], dtype=np.float64)).to(cur.device)
            p = torch.empty((d, (d + 1) // 2), dtype=torch.float64, device=w.device)
            api.cp_transfer_build(ctx, w, p)
            ph.append(p)
            wd.append(w)
        cdims = tuple((d + 1) // 2 if ph[n] is not None else d for n, d in enumerate(cur.dims))
        nxt = api.DeviceTensor.empty(cdims, fp64=fp64 or prec == CP_FP64 or not fp32,
                                     fp32=fp32 or prec == CP_MIXED)
        # coarse tensors by the factored form of eq. (15) (stencil + bidiagonal solve)
        if prec == CP_MIXED:
            api.cp_restrict_factored(ctx, cur, wd, nxt, CP_MIXED)
        if nxt.z64 is not None and (cur.z64 is not None or isinstance(cur, api.SparseTensor)):
            api.cp_restrict_factored(ctx, cur, wd, nxt, CP_FP64)
        levels.append((cur, ph))
        cur = nxt
    levels.append((cur, [None] * cur.order))
    return levels


def fas_solve(ctx, levels, Z, A, fit_tol=1e-12, max_cycles=500, nu1=1, nu2=1, nuc=50, gs_iters=10,
              ic_rule=0, prec=CP_FP64, tol32=1e-9, window=1):
    """CP-FAS V-cycles (Algorithm 2) until the relative change of the exact fit is
    <= fit_tol (Section 6 caps: at most ``max_cycles`` cycles).  ``levels`` from
    :func:`build_hierarchy`; ``Z`` is the finest-level DeviceTensor.

    Mixed form: V-cycles with FP32 contractions and coarse tensors while the fit
    gains more than ``tol32`` * fit per cycle, then FP64 V-cycles (the levels
    need both the FP32 and the FP64 tensors) until the fit_tol rule holds, so
    the solve ends on the FP64 fixed point.  ``sweeps32`` / ``sweeps64`` count
    the cycles of each phase.

    CP-FAS is not a descent method: the fit of successive cycles can zigzag,
    and a single small change can be a crossing rather than convergence.
    ``window`` > 1 stops only when the last ``window`` changes are all within
    the tolerance (1: the plain rule, as the oracle's driver applies it).
    """
    torch = _torch()
    res = SolveResult()
    prev = None
    cur = prec
    small = 0
    fbuf = torch.zeros(1, dtype=torch.float64, device=Z.device)
    norm2 = float(Z.norm2.item())
    while res.sweeps < max_cycles:
        api.cp_fas_vcycle(ctx, levels, A, nu1=nu1, nu2=nu2, nuc=nuc, gs_iters=gs_iters, ic_rule=ic_rule,
                          prec=cur)
        fit = exact_fit(ctx, Z, A, fbuf, norm2)
        res.fits.append(fit)
        res.sweeps += 1
        if cur == CP_MIXED:
            res.sweeps32 += 1
            if prev is not None and fit - prev <= tol32 * abs(fit):
                cur = CP_FP64
        else:
            res.sweeps64 += 1
            if fit_tol and prev is not None and abs(fit - prev) <= fit_tol * abs(fit):
                small += 1
                if small >= window:
                    res.converged = True
                    break
            else:
                small = 0
        prev = fit
    res.final_fit = res.fits[-1] if res.fits else float("nan")
    return res


# ---------------------------------------------------------------------------
# Setup phase (Section 4, Algorithm 1), FMG (Algorithm 3) and the Section 6.1
# driver.  Every numeric step is a libcpamg call; the host recurses over the
# levels, packs factor sets side by side (device copies) and applies the
# stopping rules.
# ---------------------------------------------------------------------------
SETUP_NU1, SETUP_NU2, SETUP_NUC = 5, 5, 100   # Table 1


def grad_norm(ctx, Z, A):
    """g of eq. (30) at A (device call, read back)."""
    torch = _torch()
    g = torch.zeros(1, dtype=torch.float64, device=Z.device)
    api.cp_objective(ctx, Z, A, exact=True, g=g)
    return float(g.item())


def _pack(sets):
    """One factor set holding `sets` (equal rank) side by side as column groups."""
    torch = _torch()
    mats = [torch.cat([s.mats[n] for s in sets], dim=1).contiguous() for n in range(len(sets[0].mats))]
    return api.DeviceFactors(mats)


def _unpack(packed, k, R, dst):
    for n, m in enumerate(dst.mats):
        m.copy_(packed.mats[n][:, k * R:(k + 1) * R])


def _relax_groups(ctx, Z, sets, sweeps):
    """`sweeps` ALS sweeps (Section 3, normalized, eq. (10)) on each factor set,
    all sets sharing every pass over Z as column groups (cp_als_batched)."""
    if sweeps <= 0 or not sets:
        return
    if isinstance(Z, api.SparseTensor):
        # the batched solve takes dense tensors only: one set after the other
        for s in sets:
            api.cp_als_sweep(ctx, Z, s, None, sweeps, CP_SOLVE_CHOL, 10, True, CP_FP64)
        return
    R = sets[0].rank
    P = _pack(sets)
    api.cp_als_batched(ctx, [(Z, P)], len(sets), prec=CP_FP64, tol64=0.0, max_sweeps=sweeps, chunk=sweeps)
    for k, s in enumerate(sets):
        _unpack(P, k, R, s)


def _level_weights(ctx, Z, fit_sets, Ic):
    """LS weights (device, cp_interp_weights) and P^ (cp_transfer_build) of every
    coarsened mode from the column groups `fit_sets`."""
    torch = _torch()
    P = _pack(fit_sets)
    phat, weights = [None] * Z.order, [None] * Z.order
    for n in Ic:
        d = Z.dims[n]
        w = torch.empty((d, 2), dtype=torch.float64, device=Z.device)
        api.cp_interp_weights(ctx, Z, P, len(fit_sets), len(fit_sets), n, w)
        ph = torch.empty((d, (d + 1) // 2), dtype=torch.float64, device=w.device)
        api.cp_transfer_build(ctx, w, ph)
        phat[n], weights[n] = ph, w
    return phat, weights


def _restrict_tensor(ctx, Z, weights):
    """Coarse tensor eq. (15) in factored form from the interpolation weights."""
    cdims = tuple((d + 1) // 2 if weights[n] is not None else d for n, d in enumerate(Z.dims))
    Zc = api.DeviceTensor.empty(cdims, fp64=True)
    api.cp_restrict_factored(ctx, Z, weights, Zc, CP_FP64)
    torch = _torch()
    Zc.norm2 = torch.zeros(1, dtype=torch.float64, device=Z.device)
    api.cp_norm2(ctx, Zc, Zc.norm2)
    return Zc


def _restrict_factors(ctx, phat, A):
    """A~_c^(n) = R^^(n) A^(n) (eq. (21)); a copy for modes that are not coarsened."""
    torch = _torch()
    mats = []
    for n, a in enumerate(A.mats):
        if phat[n] is None:
            mats.append(a.clone())
        else:
            out = torch.empty(((a.shape[0] + 1) // 2, a.shape[1]), dtype=torch.float64, device=a.device)
            api.cp_restrict_factor(ctx, phat[n], a, out)
            mats.append(out)
    return api.DeviceFactors(mats)


def _prolong_into(ctx, phat, Ac, A):
    """A^(n) = P^^(n) A_c^(n) (eq. (22)); a copy for modes that are not coarsened."""
    for n, (ac, a) in enumerate(zip(Ac.mats, A.mats)):
        if phat[n] is None:
            a.copy_(ac)
        else:
            api.cp_prolong(ctx, phat[n], ac, None, a)


def _coarsened(Z, coarsest):
    return [n for n, d in enumerate(Z.dims) if d > coarsest[n]]


def mult_vcycle(ctx, Z, A, tfms, coarsest, first_cycle, nu1=SETUP_NU1, nu2=SETUP_NU2, nuc=SETUP_NUC,
                levels_out=None, weights_out=None):
    """Algorithm 1 (CP-AMG-mult) from level Z: nu1 ALS sweeps on every TFM block
    and on the BFMs (one multi-block pass per sweep), LS weights from the TFMs
    (and, after the first cycle, the BFMs), P^ of every coarsened mode, the
    coarse tensor and restricted blocks, recursion, coarse-grid correction
    A = P^ A^_c and nu2 ALS sweeps.  On the coarsest level: nuc ALS sweeps on
    the BFMs.  A (BFMs) and the fine TFMs are updated in place; returns the level
    list [(tensor, phat per mode)] for cp_fas_vcycle (finest first)."""
    if levels_out is None:
        levels_out, weights_out = [], []
    N = Z.order
    Ic = _coarsened(Z, coarsest)
    if not Ic:
        api.cp_als_sweep(ctx, Z, A, None, nuc, CP_SOLVE_CHOL, 10, True, CP_FP64)
        levels_out.append((Z, [None] * N))
        weights_out.append([None] * N)
        return levels_out, weights_out
    _relax_groups(ctx, Z, list(tfms) + [A], nu1)
    phat, weights = _level_weights(ctx, Z, list(tfms) + ([] if first_cycle else [A]), Ic)
    levels_out.append((Z, phat))
    weights_out.append(weights)
    Zc = _restrict_tensor(ctx, Z, weights)
    Ac = _restrict_factors(ctx, phat, A)
    tfms_c = [_restrict_factors(ctx, phat, T) for T in tfms]
    mult_vcycle(ctx, Zc, Ac, tfms_c, coarsest, first_cycle, nu1, nu2, nuc, levels_out, weights_out)
    _prolong_into(ctx, phat, Ac, A)
    api.cp_als_sweep(ctx, Z, A, None, nu2, CP_SOLVE_CHOL, 10, True, CP_FP64)
    return levels_out, weights_out


def setup_phase(ctx, Z, A, tfms, coarsest, max_cycles=5, check_after=3, eps=0.1, **mult):
    """Setup cycles of Section 6.1: Algorithm 1 cycles until g_new > (1 - eps) g_old
    (eq. (32)), checked once `check_after` cycles have completed, at most
    `max_cycles`.  A and the TFMs are updated in place.  Returns (levels, weights,
    g history)."""
    g_old = grad_norm(ctx, Z, A)
    levels = weights = None
    hist = []
    for c in range(max_cycles):
        levels, weights = mult_vcycle(ctx, Z, A, tfms, coarsest, first_cycle=(c == 0), **mult)
        g_new = grad_norm(ctx, Z, A)
        hist.append(g_new)
        if c + 1 >= check_after and g_new > (1.0 - eps) * g_old:
            break
        g_old = g_new
    return levels, weights, hist


def down_sweep(ctx, Z, A_boot, tfms, coarsest, nu1=SETUP_NU1, use_bfm=True):
    """Downward half of Algorithm 1 (the rebuild of Section 6.1): the TFMs are
    relaxed (nu1 ALS sweeps per level), the boot factors only restricted, and
    the transfer operators rebuilt.  The fine TFMs are updated in place; the boot
    factors are left unchanged.  Returns (levels, weights)."""
    levels, weights = [], []
    cur, B, T = Z, A_boot, list(tfms)
    while True:
        N = cur.order
        Ic = _coarsened(cur, coarsest)
        if not Ic:
            levels.append((cur, [None] * N))
            weights.append([None] * N)
            break
        _relax_groups(ctx, cur, T, nu1)   # on the finest level: the caller's TFMs, in place
        phat, w = _level_weights(ctx, cur, T + ([B] if use_bfm else []), Ic)
        levels.append((cur, phat))
        weights.append(w)
        B = _restrict_factors(ctx, phat, B)
        T = [_restrict_factors(ctx, phat, t) for t in T]
        cur = _restrict_tensor(ctx, cur, w)
    return levels, weights


def fmg_cycle(ctx, levels, A_coarse, nu=SETUP_NUC, **fas):
    """Algorithm 3 (FMG-CP-FAS): nu ALS sweeps on the coarsest level from
    A_coarse, then, level by level towards the finest, A = P^ A_c and one CP-FAS
    V-cycle with F = 0 from that level.  Returns the finest-level factors."""
    L = len(levels)
    A = A_coarse
    api.cp_als_sweep(ctx, levels[L - 1][0], A, None, nu, CP_SOLVE_CHOL, 10, True, CP_FP64)
    torch = _torch()
    for l in range(L - 1, 0, -1):
        Zf, phat = levels[l - 1]
        Af = api.DeviceFactors([torch.empty((d, A.rank), dtype=torch.float64, device=A.mats[0].device)
                                for d in Zf.dims])
        _prolong_into(ctx, phat, A, Af)
        api.cp_fas_vcycle(ctx, levels[l - 1:], Af, **fas)
        A = Af
    return A


def solve_phase(ctx, Z, A, levels, tfms, coarsest, tau=1e-10, max_cycles=500, stagnation_after=5,
                nu1_setup=SETUP_NU1, **fas):
    """Solve cycles of Section 6.1: CP-FAS V-cycles until g < tau; once five
    cycles have completed, a cycle with g_new >= g_old is discarded and the
    transfer operators are rebuilt by one down-sweep from the previous iterate
    (once).  A is updated in place.  Returns (levels, g history, rebuilt).

    A cycle whose g is not finite (the cycle diverged) is discarded at any
    point: it triggers the one rebuild, or ends the phase once that is spent,
    leaving A at the last finite iterate."""
    g_old = grad_norm(ctx, Z, A)
    rebuilt = False
    hist = []
    for c in range(max_cycles):
        An = A.clone()
        api.cp_fas_vcycle(ctx, levels, An, **fas)
        g_new = grad_norm(ctx, Z, An)
        if not math.isfinite(g_new):
            if rebuilt:
                break
            levels, _ = down_sweep(ctx, Z, A, tfms, coarsest, nu1=nu1_setup)
            rebuilt = True
            continue
        if c + 1 > stagnation_after and g_new >= g_old and not rebuilt:
            levels, _ = down_sweep(ctx, Z, A, tfms, coarsest, nu1=nu1_setup)
            rebuilt = True
            continue
        _copy_factors(A, An)
        g_old = g_new
        hist.append(g_new)
        if g_new < tau:
            break
    return levels, hist, rebuilt


def multilevel_fmg(ctx, Z, A, tfms, coarsest, coarse_start, tau=1e-10, max_cycles=500, fmg_nu=SETUP_NUC,
                   setup=None, fas=None):
    """'Multilevel + FMG' of Section 6.1: setup cycles (stopped by eq. (32)), one
    FMG-CP-FAS cycle (Algorithm 3) from `coarse_start` on the coarsest level whose
    result replaces the boot factors, one down-sweep rebuild of the transfer
    operators with those boot factors (test blocks relaxed, boot factors not),
    then CP-FAS solve cycles until g < tau.  A (the boot factors) and the TFMs are
    updated in place; `coarse_start` is overwritten by the coarsest-level ALS.
    Returns a dict: g after each setup cycle, after the FMG cycle and after each
    kept solve cycle, whether the solve phase rebuilt its operators, the level
    count and the iteration count (setup plus solve cycles)."""
    setup = dict(setup or {})
    fas = dict(fas or {})
    levels, _, shist = setup_phase(ctx, Z, A, tfms, coarsest, **setup)
    Af = fmg_cycle(ctx, levels, coarse_start, nu=fmg_nu, **fas)
    _copy_factors(A, Af)
    g_fmg = grad_norm(ctx, Z, A)
    nu1 = setup.get("nu1", SETUP_NU1)
    levels, _ = down_sweep(ctx, Z, A, tfms, coarsest, nu1=nu1)
    levels, hist, rebuilt = solve_phase(ctx, Z, A, levels, tfms, coarsest, tau, max_cycles,
                                        nu1_setup=nu1, **fas)
    return dict(setup=shist, fmg=g_fmg, solve=hist, rebuilt=rebuilt, levels=len(levels),
                iterations=len(shist) + len(hist))


def als_solve_g(ctx, Z, A, tau=1e-10, max_sweeps=10000, chunk=32, prec=CP_FP64):
    """Standalone ALS stopped by eq. (31): g < tau, with g of eq. (30) evaluated
    on the device after every sweep and read back once per chunk.  When the rule
    holds after sweep j of a chunk, the factors are put back as they were before
    the chunk and exactly j sweeps are run again (the kernels are deterministic).
    Returns (sweeps, g history)."""
    torch = _torch()
    dev = A.mats[0].device
    gbuf = torch.zeros(chunk, dtype=torch.float64, device=dev)
    snap = A.clone()
    sweeps, hist = 0, []
    while sweeps < max_sweeps:
        k = min(chunk, max_sweeps - sweeps)
        _copy_factors(snap, A)
        for j in range(k):
            api.cp_als_sweep(ctx, Z, A, None, 1, CP_SOLVE_CHOL, 10, True, prec)
            api.cp_objective(ctx, Z, A, exact=True, g=gbuf[j:j + 1])
        gv = gbuf[:k].cpu().numpy()
        hit = next((j for j in range(k) if gv[j] < tau), None)
        if hit is None:
            hist.extend(float(x) for x in gv)
            sweeps += k
            continue
        hist.extend(float(x) for x in gv[:hit + 1])
        sweeps += hit + 1
        if hit + 1 < k:
            _copy_factors(A, snap)
            api.cp_als_sweep(ctx, Z, A, None, hit + 1, CP_SOLVE_CHOL, 10, True, prec)
        break
    return sweeps, hist


def multilevel(ctx, Z, A, tfms, coarsest, tau=1e-10, max_cycles=500, setup=None, fas=None):
    """'Multilevel' of Section 6.1 (no FMG): setup cycles stopped by eq. (32),
    then CP-FAS solve cycles from the setup's boot factors on the setup's levels
    until g < tau, with the one stagnation rebuild.  A and the TFMs are updated
    in place.  Returns the dict of `multilevel_fmg` without 'fmg'."""
    setup = dict(setup or {})
    fas = dict(fas or {})
    levels, _, shist = setup_phase(ctx, Z, A, tfms, coarsest, **setup)
    levels, hist, rebuilt = solve_phase(ctx, Z, A, levels, tfms, coarsest, tau, max_cycles,
                                        nu1_setup=setup.get("nu1", SETUP_NU1), **fas)
    return dict(setup=shist, solve=hist, rebuilt=rebuilt, levels=len(levels),
                iterations=len(shist) + len(hist))


def tune_batched(ctx, problems, restarts, prec, candidates=(48, 96, 192, 384, 768), sweeps=8,
                 near=0.03):
    """Launch-tile tuner of the batched solve: times `sweeps` sweeps of the whole
    batch (every restart running: no stopping rule) for each candidate tensor
    KiB per streaming workgroup, on copies of the factors, and returns
    (chosen wg_kib, {wg_kib: seconds}).

    The choice is the smallest tile within ``near`` (relative) of the fastest:
    the timed sweeps have every restart active, while the solve spends much of
    its time with fewer problems left, where smaller tiles spread what remains
    over more workgroups."""
    torch = _torch()
    times = {}
    work = [(Z, A.clone()) for Z, A in problems]
    api.cp_als_batched(ctx, work, restarts, prec=prec, tol32=0.0, tol64=0.0, max_sweeps=2, chunk=2,
                       wg_kib=candidates[0])
    for kib in candidates:
        work = [(Z, A.clone()) for Z, A in problems]
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        api.cp_als_batched(ctx, work, restarts, prec=prec, tol32=0.0, tol64=0.0, max_sweeps=sweeps,
                           chunk=sweeps, wg_kib=kib)
        e1.record(st)
        torch.cuda.synchronize()
        times[kib] = e0.elapsed_time(e1) / 1e3
    return pick_tile(times, near), times


def pick_tile(times, near=0.03):
    """Smallest key of {tile: seconds} whose time is within ``near`` of the fastest."""
    fastest = min(times.values())
    return min(k for k, t in times.items() if t <= fastest * (1.0 + near))

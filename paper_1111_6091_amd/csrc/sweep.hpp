// Per-mode bookkeeping of an ALS / BNGS sweep, done by one workgroup.
//
// Normalization eq. (10) is carried lazily: the library keeps, per mode m, a
// column scale sigma^(m) with  (normalized factor) = sigma^(m) (.) (stored
// factor), and every update works in normalized coordinates.  This workgroup
// (the extra first workgroup of each MTTKRP launch, hidden under the tensor
// stream, or the finalize kernel at the end of a call) refreshes the Gram of
// the factor updated last, closes a sweep (fused objective, new normalization
// scales) and prepares Gamma^(n) (Cholesky factor, pseudoinverse, or Gamma
// itself for Gauss-Seidel) together with the column scales of the update.
#pragma once

#include "internal.hpp"
#include "smallla.hpp"

namespace cpamg {


// Block-wide sum of one double per thread; result valid in every thread.
__device__ inline double wg_sum(double v, double* sred) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = (blockDim.x + 63) / 64;
  for (int w = 0; w < nw; ++w) s += sred[w];
  return s;
}

// U (LDS, R*R) = A^T A for A (I x R row-major, global) on the matrix cores:
// v_mfma_f64_16x16x4f64 over blocks of 4 rows, lane l supplying row 4b + l/16,
// column 16t + l%16 as both operands of a diagonal tile (16x16 output tiles
// (ta, tb), ta <= tb, mirrored).  Wave w takes the row blocks w, w + 4, ...,
// Q of them per round of loads; the four wave sums are added in wave order
// (W4: 1024 doubles of LDS scratch: one barrier; NULL: a barrier per wave).
// RMAX <= 16: the diagonal tile only (one accumulator).
// gram_first_loads issues the first round of tile (0, 0) early (into pre), so
// that it shares a round trip with other loads; gram_mfma consumes it.
template <int Q>
__device__ inline void gram_first_loads(const double* __restrict__ A, int64_t I, int R, double (&pre)[Q]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t row = (int64_t)(wave + 4 * q) * 4 + kq;
    pre[q] = (row < I && r16 < R) ? A[row * R + r16] : 0.0;
  }
}

template <int Q, int RMAX>
__device__ inline void gram_mfma(const double* __restrict__ A, int64_t I, int R, double* U,
                                 const double (&pre)[Q], double* W4) {
  typedef double d4v __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int nt = RMAX <= 16 ? 1 : (R + 15) / 16;   // R <= RMAX
  const int64_t nblk = (I + 3) / 4;
  for (int ta = 0; ta < nt; ++ta)
    for (int tb = ta; tb < nt; ++tb) {
      d4v acc = {0.0, 0.0, 0.0, 0.0};
      const int ca = ta * 16 + r16, cb = tb * 16 + r16;
      int64_t b0 = wave;
      if (ta == 0 && tb == 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(pre[q], pre[q], acc, 0, 0, 0);
        b0 += 4 * Q;
      }
      if (RMAX <= 16 || ta == tb) {
        for (; b0 < nblk; b0 += 4 * Q) {
          double va[Q];
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const int64_t row = (b0 + 4 * q) * 4 + kq;
            va[q] = (row < I && ca < R) ? A[row * R + ca] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < Q; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[q], va[q], acc, 0, 0, 0);
        }
      } else {
        constexpr int Q2 = Q / 2;
        for (; b0 < nblk; b0 += 4 * Q2) {
          double va[Q2], vb[Q2];
#pragma unroll
          for (int q = 0; q < Q2; ++q) {
            const int64_t row = (b0 + 4 * q) * 4 + kq;
            const bool okr = row < I;
            va[q] = (okr && ca < R) ? A[row * R + ca] : 0.0;
            vb[q] = (okr && cb < R) ? A[row * R + cb] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < Q2; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[q], vb[q], acc, 0, 0, 0);
        }
      }
      if (W4) {
        // D(m, n), m = 16 ta + kq + 4 v, n = 16 tb + r16: every wave parks its
        // tile in its own slot of W4 (4 x 256 doubles), one barrier, then the
        // four tiles are added in wave order
#pragma unroll
        for (int v = 0; v < 4; ++v) W4[wave * 256 + (kq + 4 * v) * 16 + r16] = acc[v];
        __syncthreads();
        {
          const int m16 = tid >> 4, n16 = tid & 15;
          const int m = ta * 16 + m16, n = tb * 16 + n16;
          if (m < R && n < R) {
            const double val = ((W4[tid] + W4[256 + tid]) + W4[512 + tid]) + W4[768 + tid];
            U[m * R + n] = val;
            if (ta != tb) U[n * R + m] = val;
          }
        }
        __syncthreads();
      } else {
        // the waves add their tiles into U one after the other (no scratch)
        for (int w = 0; w < 4; ++w) {
          if (wave == w) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int m = ta * 16 + kq + 4 * v, n = tb * 16 + r16;
              if (m < R && n < R) {
                const double val = w == 0 ? acc[v] : U[m * R + n] + acc[v];
                U[m * R + n] = val;
                if (ta != tb) U[n * R + m] = val;
              }
            }
          }
          __syncthreads();
        }
      }
    }
}

// Gamma (in G, LDS, left unchanged; block-diagonal over `groups` column groups)
// for the ALS update: the inverse W = L^-1 of its Cholesky factor (kind 0,
// Gamma^-1 = W^T W, factored block by block) or, when a block fails the
// factorization test, the pseudoinverse (kind 1; in GROUPED kernels block by
// block, each block with its own threshold) is written to out[0..R*R)
// (global), with no barrier after these stores.  S, V, P: LDS scratch of R*R
// each.  RMAX: the largest rank bucket the calling kernel instantiates; LDSV:
// factor with the rows in LDS instead of registers.
template <int RMAX, bool LDSV, bool GROUPED>
__device__ __forceinline__ void gamma_factor(double* G, int R, int groups, double* out, int32_t* kind,
                                             uint32_t* flags, double* S, double* V, double* P) {
  const int fail = wg_chol_inverse<RMAX, LDSV, GROUPED>(G, R, groups, S, P);
  if (!fail) {
    for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) out[idx] = S[idx];
    if (threadIdx.x == 0) *kind = 0;
  } else {
    int zero = 0;
    if (GROUPED && groups > 1) {
      // block by block, each with its own size and largest eigenvalue in the
      // dropping threshold (as a restart solved on its own): a restart whose
      // Gamma is small in scale keeps its eigenvalues next to a singular one
      const int n = R / groups;
      for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x)
        if (idx / R / n != idx % R / n) out[idx] = 0.0;
      double* Gc = V + n * n;   // compact copy of the block (V holds R*R >= 4 n*n)
      for (int g = 0; g < groups; ++g) {
        for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x)
          Gc[idx] = G[(g * n + idx / n) * R + g * n + idx % n];
        __syncthreads();
        zero |= wg_pinv(Gc, n, S, V, P);
        for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x)
          out[(g * n + idx / n) * R + g * n + idx % n] = P[idx];
        __syncthreads();
      }
    } else {
      zero = wg_pinv(G, R, S, V, P);
      for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) out[idx] = P[idx];
    }
    if (threadIdx.x == 0) {
      *kind = 1;
      atomicOr(flags, zero ? (CP_FLAG_PINV_FALLBACK | CP_FLAG_NOT_SPD) : CP_FLAG_PINV_FALLBACK);
    }
  }
}


// The bookkeeping state (the column scales, and the stored Grams when they
// are staged) into LDS in two steps, so that its loads share one round trip
// with the first Gram operands: prep_issue loads up to K values per thread
// (the address clamped into the state, no branch around a load), prep_store
// writes them to sS / sGr and copies any remainder beyond K * kThreads values
// in a loop.  The caller's barrier follows.  L = n1 + staged Gram entries.
template <int K>
__device__ __forceinline__ void prep_issue(const double* sigma, const double* grams, int n1, int L,
                                           double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    v[k] = 0.0;
    if (k * kThreads < L) {   // uniform
      const int j = min((int)threadIdx.x + k * kThreads, L - 1);
      const double* src = j < n1 ? sigma + j : grams + (j - n1);
      v[k] = *src;
    }
  }
}

template <int K>
__device__ __forceinline__ void prep_store(const double* sigma, const double* grams, int n1, int L,
                                           const double (&v)[K], double* sS, double* sGr) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int idx = threadIdx.x + k * kThreads;
    if (k * kThreads < L && idx < L) {
      if (idx < n1) sS[idx] = v[k];
      else sGr[idx - n1] = v[k];
    }
  }
  for (int idx = threadIdx.x + K * kThreads; idx < L; idx += kThreads) {
    if (idx < n1) sS[idx] = sigma[idx];
    else sGr[idx - n1] = grams[idx - n1];
  }
}

// Stopping rules of a batched solve, applied by thread 0 after the sweep that
// just ended (fits[g] of each group); see BatchRule.
__device__ inline void batch_rules(BatchState* st, const BatchRule& ru, const double* fits, int NG) {
  const int idx = st->sweep;   // index of the sweep that just ended, within the phase
  bool any = false;
  for (int g = 0; g < NG; ++g) {
    if (st->frozen[g]) continue;
    const double fit = fits[g];
    st->sweeps[ru.phase][g] += 1;
    bool stop = st->sweeps[0][g] + st->sweeps[1][g] >= ru.max_sweeps;
    if (ru.phase == 0) {
      const int w = idx % ru.window;
      if (w == 0) st->fit_win[g] = fit;
      else if (w == ru.window - 1 && (fit - st->fit_win[g]) / (ru.window - 1) <= ru.tol32 * fabs(fit))
        stop = true;
    } else {
      const double fp = st->fit_prev[g];
      if (fp == fp && fabs(fit - fp) <= ru.tol64 * fabs(fit)) stop = true;
    }
    st->fit_prev[g] = fit;
    st->fit[g] = fit;
    if (stop) st->frozen[g] = 1;
    else any = true;
  }
  st->sweep = idx + 1;
  st->active = any ? 1 : 0;
  if (!any && ru.phase == 0) {
    // every restart left the FP32 phase: the problem goes on with FP64 sweeps
    // at once (every restart at least one, then the FP64 rule and the cap)
    st->phase = 1;
    st->sweep = 0;
    for (int g = 0; g < NG; ++g) {
      st->frozen[g] = 0;
      st->fit_prev[g] = __builtin_nan("");
    }
    st->active = 1;
  }
}

// End of a sweep, by one thread: the objective values into the history and the
// stopping rules of a batched solve.
__device__ __forceinline__ void close_sweep(const PrepArgs& a, BatchState* st, const double* sfv,
                                            const double* sfit, int NG, bool want_f) {
  if (a.f_slot && want_f)
    for (int g = 0; g < NG; ++g) a.f_slot[g] = sfv[g];
  if (st) batch_rules(st, *a.rule, sfit, NG);
}

// The bookkeeping step; smem: a.lds doubles of LDS.  LK: global loads in
// flight per thread (8 where it shares a kernel with the streaming path, whose
// register budget it must not raise; 16 in the standalone kernels).  With finalize set,
// the pending scales are applied to the stored factors and reset instead of
// preparing an update.  With a.groups > 1 the R columns form independent
// groups: Gamma is block-diagonal, f is evaluated per group, and in a batched
// solve (a.st) frozen groups are neither renormalized nor updated; GROUPED
// (the batched kernels) factors such a Gamma block by block.
template <int LK = 8, int RMAX = 32, bool GROUPED = false>
__device__ inline void sweep_prep(const PrepArgs& a, double* smem, bool finalize) {
  __shared__ double sred[8];
  __shared__ double sfit[kMaxGroups];
  __shared__ double sfv[kMaxGroups];
  // Gram scratch (the four wave tiles) only in the standalone kernels (LK = 16):
  // inside a streaming kernel it would raise every workgroup's LDS and registers
  double* sW4 = nullptr;
  if constexpr (LK == 16) {
    __shared__ double w4[4 * 256];
    sW4 = w4;
  }
  const int R = a.R, N = a.N, n = a.n, RR = R * R, tid = threadIdx.x;
  const int NG = a.groups > 1 ? a.groups : 1;
  const int Rg = R / NG;
  BatchState* st = a.st;
  const bool active = !st || (st->active && st->phase == a.run_phase);
  if (!active && !finalize) return;   // nothing left to do in this phase
  auto col_frozen = [&](int r) -> bool { return st && st->frozen[r / Rg]; };
  double* G = smem;
  double* S = G + RR;
  double* V = S + RR;
  double* P = V + RR;
  double* U = P + RR;
  double* sS = U + RR;       // sigma, N x R
  const int lds = a.lds > prep_min_doubles(N, R) ? a.lds : prep_min_doubles(N, R);
  double* sGr = prep_stage_grams(N, R, lds) ? sS + N * R : nullptr;   // stored Grams, N x R x R
  // one round trip for every global load of the step: the scales and stored
  // Grams, the first Gram operands of the factor updated last, then the
  // boundary's inner-product partials
  // (inside a streaming kernel 8 row blocks per wave and round, not 16, to keep
  // its register count)
  constexpr int GQ = LK == 8 ? 8 : 16;
  const int n1 = N * R, Lst = n1 + (sGr ? N * RR : 0);
  double pv[LK];
  prep_issue<LK>(a.sigma, a.grams, n1, Lst, pv);
  double gpre[GQ];
  if (a.p >= 0) gram_first_loads<GQ>(a.Ap, a.Ip, R, gpre);
  const bool want_f = a.boundary && active && (a.f_slot || st);
  const double ip0 = (want_f && tid < a.inner_count) ? a.inner_part[(size_t)tid * NG] : 0.0;
  const double nz2 = want_f ? *a.norm2 : 0.0;
  prep_store<LK>(a.sigma, a.grams, n1, Lst, pv, sS, sGr);
  __syncthreads();
  if (a.p >= 0) gram_mfma<GQ, RMAX>(a.Ap, a.Ip, R, U, gpre, sW4);
  // the updated factor is normalized (frozen groups kept their columns)
  if (a.p >= 0 && tid < R && !col_frozen(tid)) sS[a.p * R + tid] = 1.0;
  __syncthreads();
  auto ups = [&](int m, int idx) -> double {
    return m == a.p ? U[idx] : (sGr ? sGr[m * RR + idx] : a.grams[(size_t)m * RR + idx]);
  };
  if (a.boundary && active) {
    if (want_f) {
      // per group: f = 1/2 (||Z||^2 - 2 <A^(N), M^(N)> + 1^T (*_m Upsilon^(m)) 1),
      // in normalized coordinates (partials of blocks b = tid + kThreads j;
      // that of block tid, group 0 loaded above)
      double ipg[kMaxGroups];
#pragma unroll
      for (int g = 0; g < kMaxGroups; ++g)
        ipg[g] = g == 0 ? ip0 : ((g < NG && tid < a.inner_count) ? a.inner_part[(size_t)tid * NG + g] : 0.0);
      for (int b = tid + kThreads; b < a.inner_count; b += kThreads)
#pragma unroll
        for (int g = 0; g < kMaxGroups; ++g)
          if (g < NG) ipg[g] += a.inner_part[(size_t)b * NG + g];
      for (int g = 0; g < NG; ++g) {
        double ip = 0.0;
#pragma unroll
        for (int q = 0; q < kMaxGroups; ++q)
          if (q == g) ip = ipg[q];
        double h = 0.0;
        for (int idx = tid; idx < Rg * Rg; idx += kThreads) {
          const int r = g * Rg + idx / Rg, c = g * Rg + idx % Rg;
          double hh = 1.0;
          for (int m = 0; m < N; ++m) hh *= sS[m * R + r] * sS[m * R + c] * ups(m, r * R + c);
          h += hh;
        }
        const double inner = wg_sum(ip, sred);
        const double nrm = wg_sum(h, sred);
        if (tid == 0) {
          const double f = 0.5 * (nz2 - 2.0 * inner + nrm);
          sfv[g] = f;
          sfit[g] = 1.0 - sqrt(fmax(2.0 * f, 0.0) / nz2);
        }
      }
    }
    if (a.normalize) {
      // eq. (10): lambda_r = (prod_m ||a_r^(m)||)^(1/N); a component with a
      // zero column is left unchanged
      __syncthreads();
      if (tid < R && !col_frozen(tid)) {
        const int r = tid;
        double nr[kMaxOrder];
        bool ok = true;
        double prod = 1.0;
        for (int m = 0; m < N; ++m) {
          nr[m] = sS[m * R + r] * sqrt(ups(m, r * R + r));
          ok = ok && (nr[m] > 0.0);
          prod *= nr[m];
        }
        const double lam = pow(prod, 1.0 / N);
        if (ok)
          for (int m = 0; m < N; ++m) sS[m * R + r] *= lam / nr[m];
      }
    }
  }
  __syncthreads();
  // global stores of the step come last: a barrier after them would wait for
  // their completion
  const bool closed = a.boundary && active && tid == 0;   // a sweep ended here
  if (finalize) {
    // apply the scales to the stored factors (and shadows), LK loads in flight
    for (int m = 0; m < N; ++m) {
      double* Am = a.A[m];
      float* A32m = a.A32[m];
      const double* sm = sS + m * R;
      const int64_t cnt = a.dims[m] * R;
      for (int64_t base = 0; base < cnt; base += LK * kThreads) {
        double v[LK];
#pragma unroll
        for (int q = 0; q < LK; ++q) {
          const int64_t idx = base + tid + q * kThreads;
          v[q] = idx < cnt ? Am[idx] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < LK; ++q) {
          const int64_t idx = base + tid + q * kThreads;
          if (idx < cnt) {
            const double sc = sm[idx % R];
            if (sc != 1.0) {
              const double w = v[q] * sc;
              Am[idx] = w;
              if (A32m) A32m[idx] = (float)w;
            }
          }
        }
      }
    }
    for (int m = 0; m < N; ++m) {
      const double* sm = sS + m * R;
      for (int idx = tid; idx < RR; idx += kThreads) {
        const int r = idx / R, c = idx % R;
        a.grams[(size_t)m * RR + idx] = sm[r] * sm[c] * ups(m, idx);
      }
    }
    for (int idx = tid; idx < N * R; idx += kThreads) a.sigma[idx] = 1.0;
    if (closed) close_sweep(a, st, sfv, sfit, NG, want_f);
    return;
  }
  // Gamma^(n) in normalized coordinates, column scale of M^(n), sigma^(n)
  for (int idx = tid; idx < RR; idx += kThreads) {
    const int r = idx / R, c = idx % R;
    double g = 0.0;
    if (r / Rg == c / Rg) {   // groups never couple
      g = 1.0;
      for (int m = 0; m < N; ++m)
        if (m != n) g *= sS[m * R + r] * sS[m * R + c] * ups(m, idx);
    }
    G[idx] = g;
  }
  __syncthreads();
  if (a.solver == CP_SOLVE_GS) {
    for (int idx = tid; idx < RR; idx += kThreads) a.out[idx] = G[idx];
    if (tid == 0) *a.kind = 2;
  } else {
    // rows in registers; inside a streaming kernel, whose register count
    // (occupancy) longer rows would raise, only up to 12 entries
    gamma_factor<(LK == 8 ? 12 : RMAX), (LK == 8), GROUPED>(G, R, NG, a.out, a.kind, a.flags, S, V, P);
  }
  if (tid < R) {
    double c = 1.0;
    for (int m = 0; m < N; ++m)
      if (m != n) c *= sS[m * R + tid];
    a.out[RR + tid] = c;
    a.out[RR + R + tid] = sS[n * R + tid];
  }
  if (a.p >= 0)
    for (int idx = tid; idx < RR; idx += kThreads) a.grams[(size_t)a.p * RR + idx] = U[idx];
  for (int idx = tid; idx < N * R; idx += kThreads) a.sigma[idx] = sS[idx];
  if (closed) close_sweep(a, st, sfv, sfit, NG, want_f);
}

}  // namespace cpamg

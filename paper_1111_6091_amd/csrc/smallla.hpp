// Small dense linear algebra on R x R matrices (R <= 32) for one workgroup.
// Every thread of the workgroup must call the wg_ functions (they use
// __syncthreads); the first wave does the arithmetic, lane = matrix row.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace cpamg {

constexpr double kEps = 2.220446049250313e-16;

// Gamma^(n) = Hadamard product of grams[m], m != n  (grams: [N][R][R]).
__device__ inline void hadamard_gamma(const double* __restrict__ grams, int N, int n, int R,
                                      double* __restrict__ G /*LDS R*R*/) {
  for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
    double g = 1.0;
    for (int m = 0; m < N; ++m)
      if (m != n) g *= grams[(size_t)m * R * R + idx];
    G[idx] = g;
  }
  __syncthreads();
}

// 1/sqrt(d) for a positive normal double: the hardware estimate refined by two
// Newton-Raphson steps y <- y (3/2 - (d/2) y^2) (within an ulp or two).
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  const double h = 0.5 * d;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// W = L^-1 for the Cholesky factor L of the symmetric positive definite R x R
// matrix G (LDS, row-major), so that G^-1 = W^T W.  Wave 0, lane i holds row i
// in registers; rows and columns R..RM-1 are padded with the identity, so every
// step is straight-line code.  Element (i, j) of G and of out is at i ld + j.
//  1. Cholesky, right-looking: step k takes the pivot a_kk, forms column k of L
//     (a_ik / sqrt(a_kk)) and subtracts L_ik L_jk from the trailing entries.
//     Bad when max diag(G) <= 0 or a pivot is <= R eps max diag(G).
//  2. Rows of W in order: row k is final after step k (W_kk = 1/L_kk,
//     W_kj = -acc_kj / L_kk), then every later row i adds L_ik W_kj to its
//     accumulator acc_ij = sum_{k<i} L_ik W_kj, kept in place of L_ij.
// Values from one lane reach every lane through scalar reads (readlane), all
// issued before the updates that use them.  Writes W (zeros above the
// diagonal) to out (LDS), lane i < R writing row i, unless bad; returns bad
// (wave-uniform).
template <int RM>
__device__ __forceinline__ bool wave_chol_inverse(const double* G, int R, int ld, double* out) {
  const int lane = threadIdx.x & 63;
  double a[RM];
#pragma unroll
  for (int k = 0; k < RM; ++k) a[k] = (lane < R && k < R) ? G[lane * ld + k] : (lane == k ? 1.0 : 0.0);
  double dmax = 0.0;
#pragma unroll
  for (int k = 0; k < RM; ++k)
    if (k < R) dmax = fmax(dmax, wave_bcast(a[k], k));
  const double thr = R * kEps * dmax;
  bool bad = !(dmax > 0.0);
  double dinv = 1.0;   // 1 / L_ii of this lane's row
#pragma unroll
  for (int k = 0; k < RM; ++k) {
    if (k < R) {
      const double piv = wave_bcast(a[k], k);
      bad = bad || !(piv > thr);
      const double rs = rsqrt_nr(piv);
      if (lane == k) dinv = rs;
      const double l = a[k] * rs;
      a[k] = l;
      double lj[RM];
#pragma unroll
      for (int j = k + 1; j < RM; ++j) lj[j] = wave_bcast(l, j);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = k + 1; j < RM; ++j) a[j] = fma(-l, lj[j], a[j]);
    }
  }
#pragma unroll
  for (int k = 0; k < RM; ++k) {
    if (k < R) {
      const double dk = wave_bcast(dinv, k);
      double wk[RM];
#pragma unroll
      for (int j = 0; j < k; ++j) wk[j] = -wave_bcast(a[j], k) * dk;
      __builtin_amdgcn_sched_barrier(0);
      const double c = lane > k ? a[k] : 0.0;
#pragma unroll
      for (int j = 0; j < k; ++j) a[j] = fma(c, wk[j], a[j]);
      a[k] = c * dk;
    }
  }
  if (!bad && lane < R) {
#pragma unroll
    for (int j = 0; j < RM; ++j)
      if (j < R) out[lane * ld + j] = j < lane ? -a[j] * dinv : (j == lane ? dinv : 0.0);
  }
  return bad;
}

// The same W = L^-1 with the rows kept in LDS (for kernels whose register
// budget the form above would raise): C (LDS, R x R) takes L, out (LDS) gets W.
// Lane i works on row i; runtime loops over columns, four at a time.  The
// column-k entries another lane wrote in the same step are read after those
// writes in program order (LDS operations of a wavefront complete in order).
__device__ __forceinline__ bool wave_chol_inverse_lds(const double* G, int R, int ld, double* C, double* out) {
  const int lane = threadIdx.x & 63;
  const bool row = lane < R;
  double dmax = 0.0;
  for (int k = 0; k < R; ++k) dmax = fmax(dmax, G[k * ld + k]);
  const double thr = R * kEps * dmax;
  bool bad = !(dmax > 0.0);
  if (row)
    for (int j = 0; j < R; ++j) C[lane * ld + j] = G[lane * ld + j];
  double dinv = 1.0;
  for (int k = 0; k < R; ++k) {
    const double piv = C[k * ld + k];
    bad = bad || !(piv > thr);
    const double rs = rsqrt_nr(piv);
    if (lane == k) dinv = rs;
    const bool act = row && lane >= k;
    const double l = act ? C[lane * ld + k] * rs : 0.0;
    if (act) C[lane * ld + k] = l;
    for (int j0 = k + 1; j0 < R; j0 += 4) {
      double lj[4], cj[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = j0 + q < R ? j0 + q : R - 1;
        lj[q] = C[j * ld + k];
        cj[q] = act ? C[lane * ld + j] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (act && j0 + q < R) C[lane * ld + j0 + q] = fma(-l, lj[q], cj[q]);
    }
  }
  // rows of W: acc_ij = sum_{k<i} L_ik W_kj in out, W_kj = -acc_kj / L_kk
  if (row)
    for (int j = 0; j < R; ++j) out[lane * ld + j] = 0.0;
  for (int k = 0; k < R; ++k) {
    const double dk = wave_bcast(dinv, k);
    const bool act = row && lane > k;
    const double c = act ? C[lane * ld + k] : 0.0;
    for (int j0 = 0; j0 <= k; j0 += 4) {
      double wk[4], aj[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = j0 + q <= k ? j0 + q : k;
        const double acc = out[k * ld + j];
        wk[q] = j == k ? dk : -acc * dk;
        aj[q] = act ? out[lane * ld + j] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (act && j0 + q <= k) out[lane * ld + j0 + q] = fma(c, wk[q], aj[q]);
    }
  }
  if (row && !bad)
    for (int j = 0; j < R; ++j) {
      const double v = out[lane * ld + j];
      out[lane * ld + j] = j < lane ? -v * dinv : (j == lane ? dinv : 0.0);
    }
  return bad;
}

// The factor inverse above for every thread of the workgroup (wave 0 works),
// block by block when G is block-diagonal with `groups` equal blocks (GROUPED
// kernels only; each
// block factored and tested on its own; zeros between the blocks of out).
// Blocks are factored with the rows in registers up to RMAX entries, in LDS (C:
// work array) beyond RMAX or, with LDSV, beyond 12.  out is LDS, visible to the
// workgroup on return.  Returns 1 in every thread when a block failed the
// factorization test (out incomplete).
template <int RMAX, bool LDSV>
__device__ __forceinline__ bool chol_inverse_block(const double* G, int n, int ld, double* C, double* out) {
  if (n > RMAX || (LDSV && n > 12)) return wave_chol_inverse_lds(G, n, ld, C, out);
  if (n <= 4) return wave_chol_inverse<4>(G, n, ld, out);
  if (n <= 8) return wave_chol_inverse<8>(G, n, ld, out);
  if (n <= 10) return wave_chol_inverse<10>(G, n, ld, out);
  if (n <= 12 || RMAX <= 12) return wave_chol_inverse<12>(G, n, ld, out);
  if (RMAX <= 16 || n <= 16) return wave_chol_inverse<16>(G, n, ld, out);
  if (n <= 24) return wave_chol_inverse<RMAX <= 16 ? 16 : 24>(G, n, ld, out);
  return wave_chol_inverse<RMAX <= 16 ? 16 : 32>(G, n, ld, out);
}

template <int RMAX, bool LDSV = false, bool GROUPED = false>
__device__ __forceinline__ int wg_chol_inverse(const double* G, int R, int groups, double* out, double* C) {
  __shared__ int s_bad;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    bool bad;
    if (!GROUPED || groups <= 1) {
      bad = chol_inverse_block<RMAX, LDSV>(G, R, R, C, out);
    } else {
      // blocks of at most 8 columns in registers (the batched restarts)
      const int n = R / groups;
      if (lane < R)
        for (int j = 0; j < R; ++j)
          if (j / n != lane / n) out[lane * R + j] = 0.0;
      bad = false;
      for (int g = 0; g < groups; ++g) {
        const int o = g * n * (R + 1);
        const bool b = n <= 8 ? (n <= 4 ? wave_chol_inverse<4>(G + o, n, R, out + o)
                                        : wave_chol_inverse<8>(G + o, n, R, out + o))
                              : wave_chol_inverse_lds(G + o, n, R, C + o, out + o);
        bad = bad || b;
      }
    }
    if (lane == 0) s_bad = bad ? 1 : 0;
  }
  __syncthreads();
  return s_bad;
}

// Pseudoinverse of the symmetric PSD matrix G (R x R) by cyclic Jacobi:
// eigenvalues <= R*eps*lambda_max are dropped.  S, V, P: LDS scratch (R*R
// each); the result is written to P.  Returns 1 if every eigenvalue was dropped.
__device__ __forceinline__ int wg_pinv(const double* G, int R, double* S, double* V, double* P) {
  const int lane = threadIdx.x;
  __shared__ double s_cs[2];
  __shared__ int s_done;
  for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
    S[idx] = G[idx];
    V[idx] = (idx / R == idx % R) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 60; ++sweep) {
    if (lane == 0) {
      double off = 0.0, fro = 0.0;
      for (int i = 0; i < R; ++i)
        for (int j = 0; j < R; ++j) {
          const double v = S[i * R + j];
          fro += v * v;
          if (i != j) off += v * v;
        }
      s_done = (off <= kEps * kEps * fro * 1e-4) ? 1 : 0;
    }
    __syncthreads();
    if (s_done) break;
    for (int p = 0; p < R - 1; ++p)
      for (int q = p + 1; q < R; ++q) {
        if (lane == 0) {
          const double apq = S[p * R + q];
          double c = 1.0, s = 0.0;
          if (apq != 0.0) {
            const double theta = (S[q * R + q] - S[p * R + p]) / (2.0 * apq);
            const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
          s_cs[0] = c;
          s_cs[1] = s;
        }
        __syncthreads();
        const double c = s_cs[0], s = s_cs[1];
        if (s != 0.0) {
          if (lane < R) {  // columns p, q of S and V
            const double skp = S[lane * R + p], skq = S[lane * R + q];
            S[lane * R + p] = c * skp - s * skq;
            S[lane * R + q] = s * skp + c * skq;
            const double vkp = V[lane * R + p], vkq = V[lane * R + q];
            V[lane * R + p] = c * vkp - s * vkq;
            V[lane * R + q] = s * vkp + c * vkq;
          }
          __syncthreads();
          if (lane < R) {  // rows p, q of S
            const double spk = S[p * R + lane], sqk = S[q * R + lane];
            S[p * R + lane] = c * spk - s * sqk;
            S[q * R + lane] = s * spk + c * sqk;
          }
        }
        __syncthreads();
      }
  }
  // P = V diag(1/w) V^T over kept eigenvalues
  double lmax = 0.0;
  for (int i = 0; i < R; ++i) lmax = fmax(lmax, S[i * R + i]);
  const double thr = R * kEps * lmax;
  int kept = 0;
  for (int i = 0; i < R; ++i) kept += (S[i * R + i] > thr) ? 1 : 0;
  for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) {
    const int i = idx / R, j = idx % R;
    double acc = 0.0;
    for (int k = 0; k < R; ++k) {
      const double w = S[k * R + k];
      if (w > thr) acc += V[i * R + k] * (1.0 / w) * V[j * R + k];
    }
    P[idx] = acc;
  }
  __syncthreads();
  return kept == 0 ? 1 : 0;
}

}  // namespace cpamg

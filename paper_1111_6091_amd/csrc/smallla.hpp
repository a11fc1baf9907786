// Small dense linear algebra on R x R matrices (R <= 32) for one workgroup.
// Every thread of the workgroup must call these functions (they use
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

// In-place Cholesky factorization G = L L^T of the symmetric R x R matrix in
// LDS (row-major; the lower triangle of G becomes L, the upper triangle is left
// stale).  Returns 1 in every thread if a pivot is <= R * eps * max diag(G)
// (or the diagonal is not positive).  Wave 0 does the work: lane i keeps row i
// in registers (RM >= R columns, loops unrolled), pivots and the entries
// L(k, j) reach every lane through scalar reads (readlane).
template <int RM>
__device__ inline int wave_cholesky(double* G, int R) {
  __shared__ int s_fail;
  const int tid = threadIdx.x;
  if (tid < 64) {
    const int lane = tid;
    const bool own = lane < R;
    double g[RM];
#pragma unroll
    for (int k = 0; k < RM; ++k) g[k] = (own && k < R) ? G[lane * R + k] : 0.0;
    double dmax = 0.0;
    for (int i = 0; i < R; ++i) dmax = fmax(dmax, G[i * R + i]);
    const double thr = R * kEps * dmax;
    int fail = dmax > 0.0 ? 0 : 1;
#pragma unroll
    for (int j = 0; j < RM; ++j) {
      if (j < R && !fail) {
        const double piv = wave_bcast(g[j], j);
        if (!(piv > thr)) {
          fail = 1;
        } else {
          const double dj = sqrt(piv);
          const double l = lane == j ? dj : (lane > j ? g[j] / dj : g[j]);
          g[j] = l;
#pragma unroll
          for (int k = j + 1; k < RM; ++k) {
            if (k < R) {
              const double lk = wave_bcast(l, k);
              if (lane >= k) g[k] -= l * lk;
            }
          }
        }
      }
    }
    if (!fail && own) {
#pragma unroll
      for (int k = 0; k < RM; ++k)
        if (k < R && k <= lane) G[lane * R + k] = g[k];
    }
    if (lane == 0) s_fail = fail;
  }
  __syncthreads();
  return s_fail;
}

// The same factorization with rows kept in LDS (few registers): lane i owns
// row i; pivots and L(k, j) are broadcast through scalar reads.
__device__ inline int wave_cholesky_lds(double* G, int R) {
  __shared__ int s_fail;
  const int tid = threadIdx.x;
  if (tid < 64) {
    const int lane = tid;
    const bool own = lane < R;
    double dmax = 0.0;
    for (int i = 0; i < R; ++i) dmax = fmax(dmax, G[i * R + i]);
    const double thr = R * kEps * dmax;
    int fail = dmax > 0.0 ? 0 : 1;
    for (int j = 0; j < R && !fail; ++j) {
      const double gj = own ? G[lane * R + j] : 0.0;
      const double piv = wave_bcast(gj, j);
      if (!(piv > thr)) {
        fail = 1;
        break;
      }
      const double dj = sqrt(piv);
      const double l = lane == j ? dj : (lane > j && own ? gj / dj : 0.0);
      if (own && lane >= j) G[lane * R + j] = l;
      for (int k = j + 1; k < R; ++k) {
        const double lk = wave_bcast(l, k);
        if (own && lane >= k) G[lane * R + k] -= l * lk;
      }
    }
    if (lane == 0) s_fail = fail;
  }
  __syncthreads();
  return s_fail;
}

// REG: rows in registers (standalone bookkeeping kernels); otherwise in LDS
// (inside streaming kernels, whose register budget it must not raise).
template <bool REG>
__device__ inline int wg_cholesky(double* G, int R) {
  if (!REG) return wave_cholesky_lds(G, R);
  return R <= 16 ? wave_cholesky<16>(G, R) : wave_cholesky<32>(G, R);
}

// Pseudoinverse of the symmetric PSD matrix G (R x R) by cyclic Jacobi:
// eigenvalues <= R*eps*lambda_max are dropped.  S, V, P: LDS scratch (R*R
// each); the result is written to P.  Returns 1 if every eigenvalue was dropped.
__device__ inline int wg_pinv(const double* G, int R, double* S, double* V, double* P) {
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

// Factor Gamma^(n) for the ALS update: writes L (kind 0) or the pseudoinverse
// (kind 1) to `out` (global, R*R) and the kind to *kind.  Needs LDS scratch of
// 4*R*R doubles.
__device__ inline void gamma_prepare(const double* __restrict__ grams, int N, int n, int R,
                                     double* __restrict__ out, int32_t* __restrict__ kind,
                                     uint32_t* __restrict__ flags, double* lds) {
  double* G = lds;
  double* S = lds + R * R;
  double* V = lds + 2 * R * R;
  double* P = lds + 3 * R * R;
  hadamard_gamma(grams, N, n, R, G);
  // keep a copy of Gamma in P (the Cholesky overwrites G)
  for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) P[idx] = G[idx];
  __syncthreads();
  const int fail = wg_cholesky<false>(G, R);
  __syncthreads();
  if (!fail) {
    for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) out[idx] = G[idx];
    if (threadIdx.x == 0) *kind = 0;
  } else {
    // restore Gamma from P into G, then pseudoinverse into P
    for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) G[idx] = P[idx];
    __syncthreads();
    const int zero = wg_pinv(G, R, S, V, P);
    for (int idx = threadIdx.x; idx < R * R; idx += blockDim.x) out[idx] = P[idx];
    if (threadIdx.x == 0) {
      *kind = 1;
      atomicOr(flags, zero ? (CP_FLAG_PINV_FALLBACK | CP_FLAG_NOT_SPD) : CP_FLAG_PINV_FALLBACK);
    }
  }
  __syncthreads();
}

}  // namespace cpamg

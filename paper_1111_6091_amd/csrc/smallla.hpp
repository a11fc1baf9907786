// Small dense linear algebra on R x R matrices (R <= 32) for one workgroup.
// Every thread of the workgroup must call these functions (they use
// __syncthreads); the first wave does the arithmetic, lane = matrix row.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

// In-place Cholesky G = L L^T (row-major, lower triangle receives L).
// Returns 0 on success, 1 when a pivot is <= R*eps*max(diag G) (caller falls
// back to the pseudoinverse).  G must be restored by the caller on failure.
__device__ inline int wg_cholesky(double* G, int R) {
  __shared__ int s_fail;
  const int lane = threadIdx.x;
  if (lane == 0) s_fail = 0;
  __syncthreads();
  double dmax = 0.0;
  for (int i = 0; i < R; ++i) dmax = fmax(dmax, G[i * R + i]);
  const double thr = R * kEps * dmax;
  if (!(dmax > 0.0)) return 1;
  for (int j = 0; j < R; ++j) {
    const double piv = G[j * R + j];
    if (!(piv > thr)) return 1;   // uniform: every thread reads the same value
    const double dj = sqrt(piv);
    __syncthreads();
    if (lane > j && lane < R) G[lane * R + j] /= dj;
    __syncthreads();
    if (lane == j) G[j * R + j] = dj;
    if (lane > j && lane < R) {
      const double lij = G[lane * R + j];
      for (int k = j + 1; k <= lane; ++k) G[lane * R + k] -= lij * G[k * R + j];
    }
    __syncthreads();
  }
  return 0;
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
  const int fail = wg_cholesky(G, R);
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

// Least-squares interpolation weights of the multiplicative setup phase
// (Section 4.4, eqs. (19)-(20), Algorithm 1 step 3) for one mode.
//
// The test blocks are the column groups of one factor set: group k holds the
// R_g columns [k R_g, (k + 1) R_g) of every factor.  For the mode n being
// coarsened and each fitted group k:
//   omega_k = ||A_k^(n)||^2 / max(||G_k^(n)||^2, (1e-8 ||M_k^(n)||)^2),
//   G_k^(n) = A_k^(n) Gamma_k^(n) - M_k^(n)
// (the gradient of f at that block, Gamma_k the Hadamard product of the other
// modes' Grams restricted to the group; the floor: after an ALS sweep the
// gradient of the mode solved last vanishes identically, so its computed norm
// is rounding noise and is taken at that level instead), and for every fine
// point i (odd
// 0-based index) the weights w_i of its coarse neighbours C_i (points i - 1 and
// i + 1, the latter when it exists) minimize
//   sum_k omega_k sum_{r in group k} (u_r(i) - sum_{j in C_i} w_ij u_r(j))^2
// over the columns u_r of the fitted groups (coarse values are injections of the
// fine vectors at the coarse points).  The 1 x 1 or 2 x 2 normal equations are
// solved directly (Gaussian elimination with partial pivoting).
#include "internal.hpp"

namespace cpamg {

constexpr int kSetupThreads = 256;
constexpr double kGradFloor = 1e-8;   // ||G|| floor relative to ||M||

// One workgroup.  A: mode-n factor (I x Rt row-major, Rt = groups * Rg);
// M: its MTTKRP (I x Rt); grams: N Grams of the full factor set (Rt x Rt);
// w: I x 2 output.
__global__ __launch_bounds__(kSetupThreads) void interp_weights_kernel(
    const double* __restrict__ A, const double* __restrict__ M, const double* __restrict__ grams, int N,
    int n, int64_t I, int Rt, int Rg, int nfit, double* __restrict__ w) {
  __shared__ double s_om[kMaxGroups];
  __shared__ double s_red[3][kSetupThreads];
  __shared__ double s_gam[kMaxRank * kMaxRank];
  const int tid = threadIdx.x;
  // Gamma of the whole set (only the diagonal blocks are used)
  for (int idx = tid; idx < Rt * Rt; idx += kSetupThreads) {
    double g = 1.0;
    for (int m = 0; m < N; ++m)
      if (m != n) g *= grams[(size_t)m * Rt * Rt + idx];
    s_gam[idx] = g;
  }
  __syncthreads();
  // per group: ||A_k||^2 and ||A_k Gamma_k - M_k||^2 (rows split over threads,
  // thread sums added in thread order)
  for (int k = 0; k < nfit; ++k) {
    const int c0 = k * Rg;
    double a2 = 0.0, g2 = 0.0, m2 = 0.0;
    for (int64_t i = tid; i < I; i += kSetupThreads) {
      const double* ai = A + i * Rt;
      for (int c = 0; c < Rg; ++c) {
        double h = 0.0;
        for (int q = 0; q < Rg; ++q) h += ai[c0 + q] * s_gam[(c0 + q) * Rt + c0 + c];
        const double m = M[i * Rt + c0 + c];
        h -= m;
        g2 += h * h;
        m2 += m * m;
        a2 += ai[c0 + c] * ai[c0 + c];
      }
    }
    s_red[0][tid] = a2;
    s_red[1][tid] = g2;
    s_red[2][tid] = m2;
    __syncthreads();
    if (tid == 0) {
      double sa = 0.0, sg = 0.0, sm = 0.0;
      for (int t = 0; t < kSetupThreads; ++t) {
        sa += s_red[0][t];
        sg += s_red[1][t];
        sm += s_red[2][t];
      }
      const double fl = kGradFloor * kGradFloor * sm;
      s_om[k] = sa / (sg > fl ? sg : fl);
    }
    __syncthreads();
  }
  // normal equations per fine point
  for (int64_t i = 1 + 2 * (int64_t)tid; i < I; i += 2 * kSetupThreads) {
    const int64_t j0 = i - 1, j1 = i + 1;
    const bool two = j1 < I;
    double a11 = 0.0, a12 = 0.0, a22 = 0.0, b1 = 0.0, b2 = 0.0;
    for (int k = 0; k < nfit; ++k) {
      const double om = s_om[k];
      for (int c = k * Rg; c < (k + 1) * Rg; ++c) {
        const double x1 = A[j0 * Rt + c], y = A[i * Rt + c];
        const double x2 = two ? A[j1 * Rt + c] : 0.0;
        a11 += om * x1 * x1;
        a12 += om * x1 * x2;
        a22 += om * x2 * x2;
        b1 += om * x1 * y;
        b2 += om * x2 * y;
      }
    }
    double w1, w2 = 0.0;
    if (!two) {
      w1 = b1 / a11;
    } else if (fabs(a11) >= fabs(a12)) {
      const double l = a12 / a11;
      w2 = (b2 - l * b1) / (a22 - l * a12);
      w1 = (b1 - a12 * w2) / a11;
    } else {
      // rows swapped: [a12 a22; a11 a12] [w1 w2]^T = [b2 b1]^T
      const double l = a11 / a12;
      w2 = (b1 - l * b2) / (a12 - l * a22);
      w1 = (b2 - a22 * w2) / a12;
    }
    w[i * 2] = w1;
    w[i * 2 + 1] = w2;
  }
  for (int64_t i = 2 * (int64_t)tid; i < I; i += 2 * kSetupThreads) {
    w[i * 2] = 0.0;
    w[i * 2 + 1] = 0.0;
  }
}

hipError_t interp_weights_launch(const double* A, const double* M, const double* grams, int N, int n,
                                 int64_t I, int Rt, int Rg, int nfit, double* w, hipStream_t st) {
  hipLaunchKernelGGL(interp_weights_kernel, dim3(1), dim3(kSetupThreads), 0, st, A, M, grams, N, n, I, Rt, Rg,
                     nfit, w);
  return hipGetLastError();
}

}  // namespace cpamg

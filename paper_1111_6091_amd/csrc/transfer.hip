// Transfer operators and coarse tensors (Section 4.1, Algorithm 1/2):
//   B = P^T P, L = chol(B), P^ = P L^{-T}   (geometric coarsening, Section 4.3)
//   Zc = Z x_n P^^T  (mode-n GEMM on the matrix cores)
//   A = P^ Ac,  A += P^ (Ac - A~c),  A~c = P^^T A,  Fc = Hc + P^^T (F - H)
#include <algorithm>

#include "internal.hpp"

namespace cpamg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// P^ from interpolation weights.  For the 0-based point i: even i is coarse
// point i/2 (injection); odd i interpolates from (i-1)/2 (weight w[i][0]) and,
// when i+1 < I, from (i+1)/2 (weight w[i][1]).  B = P^T P is tridiagonal:
//   B_jj = 1 + w[2j-1][1]^2 + w[2j+1][0]^2,   B_{j,j+1} = w[2j+1][0] w[2j+1][1]
// (terms whose row does not exist or has a single neighbour vanish).
// B, then its bidiagonal Cholesky factor L (diagonal ldiag[j], subdiagonal
// lsub[j] = L_{j, j-1}; lsub[0] = 0).  Every thread of the block calls it: the
// entries of B are formed side by side (into sB, 2 Ic doubles, or read from w
// on the fly when sB is NULL), then one thread runs the sequential recurrence
// l_jj = sqrt(B_jj - l_{j,j-1}^2), l_{j+1,j} = B_{j,j+1} / l_jj with the
// entries of B eight at a time ahead of the chain; the block is synchronized
// on return.
__device__ inline double bdiag(int64_t I, const double* w, int64_t j) {
  double b = 1.0;
  if (j >= 1) b += w[(2 * j - 1) * 2 + 1] * w[(2 * j - 1) * 2 + 1];
  if (2 * j + 1 < I) b += w[(2 * j + 1) * 2 + 0] * w[(2 * j + 1) * 2 + 0];
  return b;
}
__device__ inline double boff(int64_t I, const double* w, int64_t j) {   // B_{j, j+1}
  return 2 * j + 2 < I ? w[(2 * j + 1) * 2 + 0] * w[(2 * j + 1) * 2 + 1] : 0.0;
}

__device__ inline void bidiag_chol(int64_t I, const double* __restrict__ w, double* __restrict__ ldiag,
                                   double* __restrict__ lsub, double* sB) {
  const int64_t Ic = (I + 1) / 2;
  if (sB) {
    for (int64_t j = threadIdx.x; j < Ic; j += blockDim.x) {
      sB[j] = bdiag(I, w, j);
      sB[Ic + j] = boff(I, w, j);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double prev_sub = 0.0;
    lsub[0] = 0.0;
    for (int64_t j0 = 0; j0 < Ic; j0 += 8) {
      double bd[8], bo[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t j = j0 + u;
        bd[u] = j < Ic ? (sB ? sB[j] : bdiag(I, w, j)) : 1.0;
        bo[u] = j < Ic ? (sB ? sB[Ic + j] : boff(I, w, j)) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t j = j0 + u;
        if (j >= Ic) break;
        const double ljj = sqrt(bd[u] - prev_sub * prev_sub);
        ldiag[j] = ljj;
        prev_sub = (j + 1 < Ic) ? bo[u] / ljj : 0.0;
        if (j + 1 < Ic) lsub[j + 1] = prev_sub;   // L_{j+1, j}
      }
    }
  }
  __syncthreads();
}

// LDS for the entries of B when they fit (else they are formed on the fly)
constexpr int64_t kBidiagLdsMax = 4096;   // coarse extent
inline size_t bidiag_smem(int64_t I) {
  const int64_t Ic = (I + 1) / 2;
  return Ic <= kBidiagLdsMax ? (size_t)(2 * Ic) * sizeof(double) : 0;
}

__global__ __launch_bounds__(kThreads) void transfer_kernel(int64_t I, const double* __restrict__ w,
                                                            double* __restrict__ phat,
                                                            double* __restrict__ ldiag,
                                                            double* __restrict__ lsub) {
  extern __shared__ double sB[];
  const int64_t Ic = (I + 1) / 2;
  bidiag_chol(I, w, ldiag, lsub, Ic <= kBidiagLdsMax ? sB : nullptr);
  __syncthreads();
  // row i of P^: y = L^{-1} p_i (forward substitution on the bidiagonal L)
  for (int64_t i = threadIdx.x; i < I; i += kThreads) {
    int64_t j1;
    double p1, p2 = 0.0;
    if ((i & 1) == 0) {
      j1 = i / 2;
      p1 = 1.0;
    } else {
      j1 = (i - 1) / 2;
      p1 = w[i * 2 + 0];
      if (i + 1 < I) p2 = w[i * 2 + 1];
    }
    double* out = phat + i * Ic;
    for (int64_t j = 0; j < j1; ++j) out[j] = 0.0;
    double y = p1 / ldiag[j1];
    out[j1] = y;
    for (int64_t j = j1 + 1; j < Ic; ++j) {
      const double pj = (j == j1 + 1) ? p2 : 0.0;
      y = (pj - lsub[j] * y) / ldiag[j];
      out[j] = y;
    }
  }
}

hipError_t transfer_build_launch(int64_t I, const double* w, double* phat, double* ws,
                                 hipStream_t st) {
  const int64_t Ic = (I + 1) / 2;
  hipLaunchKernelGGL(transfer_kernel, dim3(1), dim3(kThreads), bidiag_smem(I), st, I, w, phat, ws, ws + Ic);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The three products with P^ (operands of at most a few hundred rows) are
// latency-bound: each output is the sum of one dense row or column of P^
// against a factor column.  kSplit consecutive lanes share an output, lane g
// taking the terms g, g + kSplit, ... (four partial sums), and the lanes' sums
// meet in an xor tree; the order is fixed, so results are deterministic.
constexpr int kSplit = 8;

__device__ __forceinline__ double split_sum(double v) {
#pragma unroll
  for (int off = 1; off < kSplit; off <<= 1) v += __shfl_xor(v, off);
  return v;
}

inline unsigned split_blocks(int64_t outputs) {
  return (unsigned)((outputs * kSplit + 255) / 256);
}

__global__ __launch_bounds__(256) void prolong_kernel(int64_t I, int64_t Ic, int R,
                                                      const double* __restrict__ phat,
                                                      const double* __restrict__ Ac,
                                                      const double* __restrict__ Act,
                                                      double* __restrict__ A) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t o = t / kSplit;
  const int g = (int)(t % kSplit);
  const bool live = o < I * R;
  const int64_t oc = live ? o : I * R - 1;   // idle lanes still take part in the sums
  const int64_t i = oc / R;
  const int r = (int)(oc % R);
  double acc;
  if (phat) {
    const double* prow = phat + i * Ic;
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t j = g;
    for (; j + 3 * kSplit < Ic; j += 4 * kSplit)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t jj = j + u * kSplit;
        a4[u] += prow[jj] * (Act ? (Ac[jj * R + r] - Act[jj * R + r]) : Ac[jj * R + r]);
      }
    for (int u = 0; j < Ic; j += kSplit, ++u)
      a4[u] += prow[j] * (Act ? (Ac[j * R + r] - Act[j * R + r]) : Ac[j * R + r]);
    acc = split_sum((a4[0] + a4[1]) + (a4[2] + a4[3]));
  } else {
    acc = Act ? (Ac[i * R + r] - Act[i * R + r]) : Ac[i * R + r];
  }
  if (live && g == 0) A[o] = Act ? A[o] + acc : acc;
}

hipError_t prolong_launch(int64_t I, int64_t Ic, int R, const double* phat, const double* Ac,
                          const double* Act, double* A, hipStream_t st) {
  if (I * R <= 0) return hipSuccess;
  hipLaunchKernelGGL(prolong_kernel, dim3(split_blocks(I * R)), dim3(256), 0, st, I, Ic, R, phat,
                     Ac, Act, A);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void restrict_factor_kernel(int64_t I, int64_t Ic, int R,
                                                              const double* __restrict__ phat,
                                                              const double* __restrict__ A,
                                                              double* __restrict__ Ac) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t o = t / kSplit;
  const int g = (int)(t % kSplit);
  const bool live = o < Ic * R;
  const int64_t oc = live ? o : Ic * R - 1;
  const int64_t j = oc / R;
  const int r = (int)(oc % R);
  double acc;
  if (phat) {
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t i = g;
    for (; i + 3 * kSplit < I; i += 4 * kSplit)
#pragma unroll
      for (int u = 0; u < 4; ++u) a4[u] += phat[(i + u * kSplit) * Ic + j] * A[(i + u * kSplit) * R + r];
    for (int u = 0; i < I; i += kSplit, ++u) a4[u] += phat[i * Ic + j] * A[i * R + r];
    acc = split_sum((a4[0] + a4[1]) + (a4[2] + a4[3]));
  } else {
    acc = A[j * R + r];
  }
  if (live && g == 0) Ac[o] = acc;
}

hipError_t restrict_factor_launch(int64_t I, int64_t Ic, int R, const double* phat,
                                  const double* A, double* Ac, hipStream_t st) {
  if (Ic * R <= 0) return hipSuccess;
  hipLaunchKernelGGL(restrict_factor_kernel, dim3(split_blocks(Ic * R)), dim3(256), 0, st, I, Ic,
                     R, phat, A, Ac);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fas_rhs_kernel(int64_t I, int64_t Ic, int R,
                                                      const double* __restrict__ phat,
                                                      const double* __restrict__ F,
                                                      const double* __restrict__ H,
                                                      const double* __restrict__ Hc,
                                                      double* __restrict__ Fc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t o = t / kSplit;
  const int g = (int)(t % kSplit);
  const bool live = o < Ic * R;
  const int64_t oc = live ? o : Ic * R - 1;
  const int64_t j = oc / R;
  const int r = (int)(oc % R);
  double a4[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t i = g;
  for (; i + 3 * kSplit < I; i += 4 * kSplit)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t ii = i + u * kSplit;
      a4[u] += phat[ii * Ic + j] * ((F ? F[ii * R + r] : 0.0) - H[ii * R + r]);
    }
  for (int u = 0; i < I; i += kSplit, ++u)
    a4[u] += phat[i * Ic + j] * ((F ? F[i * R + r] : 0.0) - H[i * R + r]);
  const double acc = split_sum((a4[0] + a4[1]) + (a4[2] + a4[3]));
  if (live && g == 0) Fc[o] = Hc[o] + acc;
}

hipError_t fas_rhs_launch(int64_t I, int64_t Ic, int R, const double* phat, const double* F,
                          const double* H, const double* Hc, double* Fc, hipStream_t st) {
  if (Ic * R <= 0) return hipSuccess;
  hipLaunchKernelGGL(fas_rhs_kernel, dim3(split_blocks(Ic * R)), dim3(256), 0, st, I, Ic, R, phat,
                     F, H, Hc, Fc);
  return hipGetLastError();
}

__global__ void fas_rhs_identity_kernel(int64_t n, const double* F, const double* H,
                                        const double* Hc, int literal, double* Fc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const double f = F ? F[idx] : 0.0;
  Fc[idx] = literal ? f : (f - H[idx] + Hc[idx]);
}

hipError_t fas_rhs_identity_launch(int64_t count, const double* F, const double* H,
                                   const double* Hc, int literal, double* Fc, hipStream_t st) {
  hipLaunchKernelGGL(fas_rhs_identity_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     st, count, F, H, Hc, literal, Fc);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Strided batched GEMM on the matrix cores.  64x64 block tile, BK = 16, four
// waves in a 2x2 arrangement of 32x32 wave tiles (2x2 MFMA 16x16x4 tiles).
template <typename T> struct GAcc;
template <> struct GAcc<double> { typedef d4 type; };
template <> struct GAcc<float> { typedef f4 type; };

__device__ __forceinline__ d4 gmma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 gmma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void gemm_kernel(GemmDesc d) {
  typedef typename GAcc<T>::type V;
  __shared__ T As[64][17];
  __shared__ T Bs[16][65];
  const T* __restrict__ A = reinterpret_cast<const T*>(d.A);
  const T* __restrict__ B = reinterpret_cast<const T*>(d.B);
  T* __restrict__ C = reinterpret_cast<T*>(d.C);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wy = wave >> 1, wx = wave & 1;
  const int64_t bm = (int64_t)blockIdx.x * 64, bn = (int64_t)blockIdx.y * 64;
  const int64_t b = blockIdx.z;
  A += b * d.a_bs;
  B += b * d.b_bs;
  C += b * d.c_bs;
  V acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = V{0, 0, 0, 0};
  const bool a_mfast = d.a_rs == 1;   // consecutive m contiguous
  const bool b_kfast = d.b_rs == 1;   // consecutive k contiguous
  for (int64_t k0 = 0; k0 < d.K; k0 += 16) {
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      int mm, kk;
      if (a_mfast) { mm = tid % 64; kk = tid / 64 + 4 * q; }
      else { kk = tid % 16; mm = tid / 16 + 16 * q; }
      const int64_t gm = bm + mm, gk = k0 + kk;
      As[mm][kk] = (gm < d.M && gk < d.K) ? A[gm * d.a_rs + gk * d.a_cs] : T(0);
      int nn, kb;
      if (b_kfast) { kb = tid % 16; nn = tid / 16 + 16 * q; }
      else { nn = tid % 64; kb = tid / 64 + 4 * q; }
      const int64_t gn = bn + nn, gkb = k0 + kb;
      Bs[kb][nn] = (gn < d.N && gkb < d.K) ? B[gkb * d.b_rs + gn * d.b_cs] : T(0);
    }
    __syncthreads();
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      T a0 = As[wy * 32 + (lane & 15)][kk];
      T a1 = As[wy * 32 + 16 + (lane & 15)][kk];
      T b0 = Bs[kk][wx * 32 + (lane & 15)];
      T b1 = Bs[kk][wx * 32 + 16 + (lane & 15)];
      acc[0][0] = gmma(a0, b0, acc[0][0]);
      acc[0][1] = gmma(a0, b1, acc[0][1]);
      acc[1][0] = gmma(a1, b0, acc[1][0]);
      acc[1][1] = gmma(a1, b1, acc[1][1]);
    }
  }
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int v = 0; v < 4; ++v) {
        const int64_t gm = bm + wy * 32 + i * 16 + mfma_row<T>(lane >> 4, v);
        const int64_t gn = bn + wx * 32 + j * 16 + (lane & 15);
        if (gm < d.M && gn < d.N) C[gm * d.c_rs + gn * d.c_cs] = acc[i][j][v];
      }
}

hipError_t gemm_launch(const GemmDesc& d, bool fp32, hipStream_t st) {
  dim3 grid((unsigned)((d.M + 63) / 64), (unsigned)((d.N + 63) / 64), (unsigned)d.batch);
  if (fp32) hipLaunchKernelGGL(gemm_kernel<float>, grid, dim3(kThreads), 0, st, d);
  else hipLaunchKernelGGL(gemm_kernel<double>, grid, dim3(kThreads), 0, st, d);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Factored restriction along one mode: Zc = Z x_n P^^T with P^^T = L^{-1} P^T,
// applied as the interpolation stencil (y_j = z_2j + w[2j-1][1] z_2j-1 +
// w[2j+1][0] z_2j+1) followed by forward substitution with the bidiagonal L:
//   x_j = a_j x_{j-1} + c0_j z_2j-1 + c1_j z_2j + c2_j z_2j+1,
// a_j = -L_{j,j-1} / L_jj, c1_j = 1 / L_jj, c0_j = w[2j-1][1] c1_j,
// c2_j = w[2j+1][0] c1_j (zero where the neighbour does not exist): about five
// flops per coarse entry and one pass over the input.  The tensor is viewed as
// (Lead, I, Tail); a column is one (lead, tail) pair.
//   Lead >= 64 (or short columns, I <= 64): a lane per column (64 consecutive
//               columns per wave, coalesced when Lead >= 64), the recurrence
//               run down the column;
//   otherwise:  a wave per column, lanes along j: the stencil values side by
//               side, then the first-order recurrence as an inclusive scan of
//               the affine maps x -> a_j x + b_j across the wave (six
//               shuffle rounds per 64 coarse entries), carried between blocks.
// coef: Ic entries of {c0, c1, c2, a}.
struct RCoef {
  double c0, c1, c2, a;
};

// one block per coarsened mode
__global__ __launch_bounds__(kThreads) void restrict_coef_kernel(RCoefJobs jobs) {
  extern __shared__ double sB[];
  const int q = blockIdx.x;
  const int64_t I = jobs.I[q];
  const double* __restrict__ w = jobs.w[q];
  RCoef* __restrict__ coef = (RCoef*)jobs.coef[q];
  const int64_t Ic = (I + 1) / 2;
  double* ldiag = jobs.scratch[q];
  double* lsub = ldiag + Ic;
  bidiag_chol(I, w, ldiag, lsub, Ic <= kBidiagLdsMax ? sB : nullptr);
  for (int64_t j = threadIdx.x; j < Ic; j += blockDim.x) {
    const double inv = 1.0 / ldiag[j];
    RCoef c;
    c.c1 = inv;
    c.c0 = j >= 1 ? w[(2 * j - 1) * 2 + 1] * inv : 0.0;
    c.c2 = 2 * j + 1 < I ? w[(2 * j + 1) * 2 + 0] * inv : 0.0;
    c.a = j >= 1 ? -lsub[j] * inv : 0.0;
    coef[j] = c;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void restrict_cols_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                                 int64_t Lead, int64_t I, int64_t Ic, int64_t Tail,
                                                                 const RCoef* __restrict__ coef) {
  constexpr int JB = 128;   // coarse entries whose coefficients sit in LDS at a time
  __shared__ RCoef sc[JB];
  const int64_t col = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool live = col < Lead * Tail;
  const int64_t l = live ? col % Lead : 0, t = live ? col / Lead : 0;
  const T* zin = in + l + Lead * I * t;
  T* zout = out + l + Lead * Ic * t;
  double x = 0.0, zprev = 0.0;
  for (int64_t jb = 0; jb < Ic; jb += JB) {
    const int nj = (int)min((int64_t)JB, Ic - jb);
    __syncthreads();
    if (threadIdx.x < nj) sc[threadIdx.x] = coef[jb + threadIdx.x];
    __syncthreads();
    if (!live) continue;
    int k = 0;
    for (; k + 8 <= nj; k += 8) {
      double z0[8], z1[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t j = jb + k + u;
        z0[u] = (double)zin[Lead * (2 * j)];
        z1[u] = 2 * j + 1 < I ? (double)zin[Lead * (2 * j + 1)] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const RCoef c = sc[k + u];
        x = c.a * x + (c.c0 * zprev + c.c1 * z0[u] + c.c2 * z1[u]);
        zprev = z1[u];
        zout[Lead * (jb + k + u)] = (T)x;
      }
    }
    for (; k < nj; ++k) {
      const int64_t j = jb + k;
      const double z0 = (double)zin[Lead * (2 * j)];
      const double z1 = 2 * j + 1 < I ? (double)zin[Lead * (2 * j + 1)] : 0.0;
      const RCoef c = sc[k];
      x = c.a * x + (c.c0 * zprev + c.c1 * z0 + c.c2 * z1);
      zprev = z1;
      zout[Lead * j] = (T)x;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void restrict_scan_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                                 int64_t Lead, int64_t I, int64_t Ic, int64_t Tail,
                                                                 const RCoef* __restrict__ coef) {
  const int lane = threadIdx.x & 63;
  const int64_t col = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (col >= Lead * Tail) return;   // whole waves leave together
  const int64_t l = col % Lead, t = col / Lead;
  const T* zin = in + l + Lead * I * t;
  T* zout = out + l + Lead * Ic * t;
  double carry = 0.0;
  for (int64_t jb = 0; jb < Ic; jb += 64) {
    const int64_t j = jb + lane;
    double A = 1.0, B = 0.0;   // identity map for lanes past the end
    if (j < Ic) {
      const RCoef c = coef[j];
      const double zl = j >= 1 ? (double)zin[Lead * (2 * j - 1)] : 0.0;
      const double z0 = (double)zin[Lead * (2 * j)];
      const double zr = 2 * j + 1 < I ? (double)zin[Lead * (2 * j + 1)] : 0.0;
      A = c.a;
      B = c.c0 * zl + c.c1 * z0 + c.c2 * zr;
    }
    // inclusive scan of x -> A x + B over the lanes (composition: later after earlier)
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double Ap = __shfl_up(A, off);
      const double Bp = __shfl_up(B, off);
      if (lane >= off) {
        B = A * Bp + B;
        A = A * Ap;
      }
    }
    const double xj = A * carry + B;
    if (j < Ic) zout[Lead * j] = (T)xj;
    carry = __shfl(xj, 63);
  }
}

hipError_t restrict_coef_launch(const RCoefJobs& jobs, hipStream_t st) {
  size_t smem = 0;
  for (int q = 0; q < jobs.count; ++q) smem = std::max(smem, bidiag_smem(jobs.I[q]));
  hipLaunchKernelGGL(restrict_coef_kernel, dim3(jobs.count), dim3(kThreads), smem, st, jobs);
  return hipGetLastError();
}

hipError_t restrict_factored_launch(const void* in, void* out, int64_t Lead, int64_t I, int64_t Tail,
                                    const void* coef, bool fp32, hipStream_t st) {
  const int64_t Ic = (I + 1) / 2;
  const int64_t cols = Lead * Tail;
  const RCoef* c = (const RCoef*)coef;
  // short fibres (I <= 64) would leave most lanes of a per-column wave idle:
  // a lane per column there too (consecutive columns then read I apart)
  if (Lead >= 64 || I <= 64) {
    const int64_t blocks = (cols + kThreads - 1) / kThreads;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (fp32)
      hipLaunchKernelGGL(restrict_cols_kernel<float>, dim3((unsigned)blocks), dim3(kThreads), 0, st,
                         (const float*)in, (float*)out, Lead, I, Ic, Tail, c);
    else
      hipLaunchKernelGGL(restrict_cols_kernel<double>, dim3((unsigned)blocks), dim3(kThreads), 0, st,
                         (const double*)in, (double*)out, Lead, I, Ic, Tail, c);
  } else {
    const int64_t per_block = kThreads / 64;
    const int64_t blocks = (cols + per_block - 1) / per_block;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (fp32)
      hipLaunchKernelGGL(restrict_scan_kernel<float>, dim3((unsigned)blocks), dim3(kThreads), 0, st,
                         (const float*)in, (float*)out, Lead, I, Ic, Tail, c);
    else
      hipLaunchKernelGGL(restrict_scan_kernel<double>, dim3((unsigned)blocks), dim3(kThreads), 0, st,
                         (const double*)in, (double*)out, Lead, I, Ic, Tail, c);
  }
  return hipGetLastError();
}

}  // namespace cpamg

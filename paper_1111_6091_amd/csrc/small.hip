// Relaxation of a small level in one workgroup.
//
// A CP-FAS V-cycle (Algorithm 2) ends on its coarsest level with nu_c = 50
// BNGS sweeps (Table 1), and every coarse level relaxes with right-hand side F
// and Gauss-Seidel inner solves (Section 5.2).  There the tensor holds a few
// thousand entries, so one sweep is a few microseconds of arithmetic while the
// general path spends two kernel launches per mode on it.  This kernel runs all
// the sweeps of one relaxation in a single workgroup: it loads the level tensor
// into LDS once, keeps the factors, the right-hand sides, their Gram matrices
// and Gamma in LDS, and writes the factors back at the end.
//
// Per sweep and mode n (in the order of the oracle's BNGS sweep):
//   Gamma^(n) = Hadamard product of the Grams of the other modes (eq. (8)),
//   M^(n)     = Z_(n) Phi^(n) (eq. (6)-(7)), Khatri-Rao matrix never formed:
//               mode 0 contracts the fibres along mode 0 with their weights,
//               the products of the other factors; after A^(0) is updated, the
//               stage-1 tiles T0[s][r] = sum_i0 Z(i0, s) A^(0)(i0, r) serve
//               every mode >= 1.  Both mode-0 contractions are dense products
//               and run on the matrix cores (v_mfma_f64_16x16x4f64), as do
//               the Grams below,
//   A^(n)     <- gs_iters Gauss-Seidel iterations on A^(n) Gamma = M + F, r in
//               increasing order with the newest values, warm-started (the
//               division by the pivot applied as a product with its reciprocal),
//   Upsilon^(n) = A^(n)T A^(n).
// All arithmetic is FP64; an FP32 tensor is widened on load.  Sums run in a
// fixed order, so results are deterministic.
#include "internal.hpp"

namespace cpamg {

typedef double sd4 __attribute__((ext_vector_type(4)));

constexpr int kSmallThreads = 512;    // 8 waves, two per SIMD; leaves room for Gamma in registers
constexpr int kSmallWaves = kSmallThreads / 64;

// Fibre stride of the tensor in LDS: odd, so that the 16 fibres of one matrix
// core operand (one entry each) fall on different banks.
__host__ __device__ inline int64_t small_fibre_stride(int64_t I0) { return I0 | 1; }

// LDS layout (in doubles unless noted); the host computes the same offsets
struct SmallLayout {
  int64_t a, f, grams, gam, m, red, t0, dig, perm, z;   // dig: uint16, perm: int32, z: T
  int64_t bytes;
};

__host__ __device__ inline SmallLayout small_layout(const SmallDesc& d, int esz) {
  SmallLayout L{};
  int64_t sumIR = 0, imax = 0;
  for (int m = 0; m < d.N; ++m) {
    sumIR += d.dims[m] * d.R;
    imax = d.dims[m] > imax ? d.dims[m] : imax;
  }
  const int64_t RR = (int64_t)d.R * d.R;
  const int64_t S0 = d.P / d.dims[0];
  int64_t o = 0;
  L.a = o;      o += sumIR;
  L.f = o;      o += sumIR;                                // right-hand sides F (zeros when absent)
  L.grams = o;  o += d.N * RR;
  L.gam = o;    o += RR;
  L.m = o;      o += imax * d.R;
  L.red = o;    o += 128 * d.R > kSmallThreads ? 128 * d.R : kSmallThreads;   // also 8 partial 16 x R tiles or R x R Grams
  L.t0 = o;     o += S0 * d.R;
  L.dig = o;    o += (S0 * (d.N - 1) * 2 + 7) / 8;        // digits s_m of every fibre, uint16
  L.perm = o;   o += (S0 * (d.N - 1) * 4 + 7) / 8;        // fibres ordered by s_n, per mode n >= 1
  L.z = o;
  L.bytes = o * 8 + S0 * small_fibre_stride(d.dims[0]) * esz;
  return L;
}

// p[0] + p[stride] + ... + p[(count-1) stride] from LDS with four partial sums
// (fixed order), so that several loads are in flight instead of one.
__device__ __forceinline__ double sum4(const double* p, int count, int stride) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int k = 0;
  for (; k + 3 < count; k += 4) {
    s0 += p[k * stride];
    s1 += p[(k + 1) * stride];
    s2 += p[(k + 2) * stride];
    s3 += p[(k + 3) * stride];
  }
  for (; k < count; ++k) s0 += p[k * stride];
  return (s0 + s1) + (s2 + s3);
}

// Gauss-Seidel iterations on the rows i < I of X (LDS, row-major, ld R), one
// thread per row: x Gamma = b with b = M + F (both LDS),
//   x_r <- (b_r - sum_{k != r} x_k Gamma_kr) / Gamma_rr, r = 0..R-1, newest values,
// a zero pivot leaving x_r as is.  RM >= R: register arrays of exactly RM
// entries with static indices only (entries r >= R are zero and never change),
// Gamma held in registers.  The equations are scaled by the reciprocal pivots
// once; per iteration the terms of the previous iterate are formed first, side
// by side, and each new x_r is then subtracted into the pending values of the
// later components, so the serial chain per component is one product and one
// subtraction.
template <int RM, int NT>
__device__ __forceinline__ void gs_rows(double* X, const double* sM, const double* sF,
                                        const double* sG, int I, int R, int iters) {
  for (int i = threadIdx.x; i < I; i += NT) {
    // the equations scaled by the reciprocal pivots: c_r = b_r / Gamma_rr,
    // h[k][r] = Gamma_kr / Gamma_rr, so that x_r = c_r - sum_{k != r} x_k h[k][r]
    // A zero pivot (and every r >= R) gets c_r = 0, h[.][r] = 0 and keep_r =
    // 1, so that t_r = x_r: the old value stays without a select in the chain
    double x[RM], c[RM], h[RM][RM], keep[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      x[r] = r < R ? X[i * R + r] : 0.0;
      const double dg = r < R ? sG[r * R + r] : 0.0;
      const bool piv = dg != 0.0;
      keep[r] = piv ? 0.0 : 1.0;
      const double dinv = piv ? 1.0 / dg : 0.0;
      c[r] = r < R ? (sM[i * R + r] + sF[i * R + r]) * dinv : 0.0;
#pragma unroll
      for (int k = 0; k < RM; ++k) h[k][r] = (k < R && r < R) ? sG[k * R + r] * dinv : 0.0;
    }
    for (int it = 0; it < iters; ++it) {
      // t_r = c_r - (terms of the previous iterate, k > r), side by side;
      // then each new x_r enters the pending t_j, j > r (one product and
      // subtraction per step of the serial chain)
      double t[RM];
#pragma unroll
      for (int r = 0; r < RM; ++r) {
        double u = 0.0;
#pragma unroll
        for (int k = r + 1; k < RM; ++k) u += x[k] * h[k][r];
        t[r] = fma(x[r], keep[r], c[r] - u);
      }
#pragma unroll
      for (int r = 0; r < RM; ++r) {
        x[r] = t[r];
#pragma unroll
        for (int j = r + 1; j < RM; ++j) t[j] -= x[r] * h[r][j];
      }
    }
#pragma unroll
    for (int r = 0; r < RM; ++r)
      if (r < R) X[i * R + r] = x[r];
  }
}

// The same iterations for 8 < R <= 16 with plain loops over LDS (x in place
// in X): register arrays of 12 or 16 entries would push the whole kernel's
// register count into spills.
template <int NT>
__device__ __forceinline__ void gs_rows_lds(double* X, const double* sM, const double* sF,
                                            const double* sG, int I, int R, int iters) {
  for (int i = threadIdx.x; i < I; i += NT) {
    double* x = X + i * R;
    for (int it = 0; it < iters; ++it)
      for (int r = 0; r < R; ++r) {
        const double dg = sG[r * R + r];
        if (dg == 0.0) continue;
        const double dinv = 1.0 / dg;
        double t = (sM[i * R + r] + sF[i * R + r]) * dinv;
        for (int k = 0; k < R; ++k)
          if (k != r) t -= x[k] * (sG[k * R + r] * dinv);
        x[r] = t;
      }
  }
}

template <int NT>
__device__ __forceinline__ void gs_rows_any(double* X, const double* sM, const double* sF,
                                            const double* sG, int I, int R, int iters) {
  switch (R) {
    case 1: case 2: gs_rows<2, NT>(X, sM, sF, sG, I, R, iters); break;
    case 3: gs_rows<3, NT>(X, sM, sF, sG, I, R, iters); break;
    case 4: gs_rows<4, NT>(X, sM, sF, sG, I, R, iters); break;
    case 5: gs_rows<5, NT>(X, sM, sF, sG, I, R, iters); break;
    case 6: gs_rows<6, NT>(X, sM, sF, sG, I, R, iters); break;
    case 7: case 8: gs_rows<8, NT>(X, sM, sF, sG, I, R, iters); break;
    default: gs_rows_lds<NT>(X, sM, sF, sG, I, R, iters); break;
  }
}

template <typename T>
__global__ __launch_bounds__(kSmallThreads) void relax_small_kernel(SmallDesc d) {
  extern __shared__ double sm[];
  const SmallLayout L = small_layout(d, (int)sizeof(T));
  const int N = d.N, R = d.R, RR = R * R, tid = threadIdx.x;
  double* sA = sm + L.a;
  double* sF = sm + L.f;
  double* sGr = sm + L.grams;
  double* sG = sm + L.gam;
  double* sM = sm + L.m;
  double* sRed = sm + L.red;
  double* sT0 = sm + L.t0;   // stage-1 tiles T0[s][r]; during mode 0 the weights W[s][r]
  uint16_t* sDig = reinterpret_cast<uint16_t*>(sm + L.dig);   // [s][m - 1]
  int32_t* sPerm = reinterpret_cast<int32_t*>(sm + L.perm);    // [n - 1][s_n * rest + k]
  T* sZ = reinterpret_cast<T*>(sm + L.z);
  int I[kMaxOrder];
  int offA[kMaxOrder];
  int st[kMaxOrder];   // strides of modes 1..N-1 in the fibre index s
  {
    int o = 0, acc = 1;
    for (int m = 0; m < N; ++m) {
      I[m] = (int)d.dims[m];
      offA[m] = o;
      o += I[m] * R;
      if (m >= 1) {
        st[m] = acc;
        acc *= I[m];
      }
    }
  }
  const int I0 = I[0];
  const int I0p = (int)small_fibre_stride(I0);
  const int S0 = (int)(d.P / I0);
  const int lane = tid & 63, wave = tid >> 6, lc = lane & 15, lj = lane >> 4;
  const int NM = N - 1;   // modes 1..N-1
  const T* __restrict__ z = reinterpret_cast<const T*>(d.z);
  // tensor and factors into LDS (several loads in flight per thread)
  for (int64_t base = 0; base < d.P; base += 8 * kSmallThreads) {
    T v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t idx = base + tid + q * kSmallThreads;
      v[q] = idx < d.P ? z[idx] : T(0);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t idx = base + tid + q * kSmallThreads;
      if (idx < d.P) {
        const int s = (int)idx / I0;
        sZ[s * I0p + ((int)idx - s * I0)] = v[q];
      }
    }
  }
  for (int m = 0; m < N; ++m)
    for (int idx = tid; idx < I[m] * R; idx += kSmallThreads) {
      sA[offA[m] + idx] = d.A[m][idx];
      sF[offA[m] + idx] = d.F[m] ? d.F[m][idx] : 0.0;
    }
  // index tables, built once: the digits of every fibre, and for each mode
  // n >= 1 the fibres listed by their digit s_n (the other digits in
  // increasing mixed-radix order)
  for (int s = tid; s < S0; s += kSmallThreads)
    for (int m = 1; m < N; ++m) sDig[s * NM + m - 1] = (uint16_t)((s / st[m]) % I[m]);
  for (int n = 1; n < N; ++n) {
    const int rest = S0 / I[n];
    int32_t* perm = sPerm + (n - 1) * S0;
    for (int j = tid; j < S0; j += kSmallThreads) {
      const int i = j / rest;
      int k = j - i * rest;
      int s = i * st[n];
      for (int m = 1; m < N; ++m) {
        if (m == n) continue;
        s += (k % I[m]) * st[m];
        k /= I[m];
      }
      perm[j] = s;
    }
  }
  __syncthreads();
  // Gram of mode m from the LDS factor on the matrix cores: A^T A as products
  // of the 16-column tile with itself, the rows four per step.  Up to 64 rows
  // one wave forms it alone; above that every wave takes a block of rows and
  // the wave tiles are added in wave order (every thread calls it)
  auto gram = [&](int m) {
    const double* a = sA + offA[m];
    const int Im = I[m];
    const int rc = lc < R ? lc : R - 1;
    const bool one = Im <= 64;
    const int chunk = one ? Im : ((Im + kSmallWaves - 1) / kSmallWaves + 15) & ~15;
    const int sb = one ? 0 : wave * chunk;
    const int se = sb + chunk < Im ? sb + chunk : Im;
    if (!one || wave == 0) {
      sd4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int k0 = sb; k0 < se; k0 += 16) {
        double av[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int kc = k0 + 4 * u + lj < Im ? k0 + 4 * u + lj : Im - 1;
          av[u] = a[kc * R + rc];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double v = (k0 + 4 * u + lj < se && lc < R) ? av[u] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc, 0, 0, 0);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = lj + 4 * v;
        if (row < R && lc < R) {
          if (one) sGr[m * RR + row * R + lc] = acc[v];
          else sRed[wave * RR + row * R + lc] = acc[v];
        }
      }
    }
    if (!one) {
      __syncthreads();
      if (tid < RR) sGr[m * RR + tid] = sum4(sRed + tid, kSmallWaves, RR);
      __syncthreads();
    }
  };
  for (int m = 0; m < N; ++m) gram(m);
  __syncthreads();

  for (int sweep = 0; sweep < d.nsweeps; ++sweep) {
    for (int n = 0; n < N; ++n) {
      // Gamma^(n)
      for (int idx = tid; idx < RR; idx += kSmallThreads) {
        double g = 1.0;
        for (int m = 0; m < N; ++m)
          if (m != n) g *= sGr[m * RR + idx];
        sG[idx] = g;
      }
      if (n == 0) {
        // weights W[s][r] = prod_{m >= 1} A^(m)(s_m, r) of every fibre, four
        // entries per thread at a time so that their loads overlap
        for (int base = tid; base < S0 * R; base += 4 * kSmallThreads) {
          double w[4] = {1.0, 1.0, 1.0, 1.0};
          int sx[4], rx[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int idx = base + u * kSmallThreads < S0 * R ? base + u * kSmallThreads : S0 * R - 1;
            sx[u] = idx / R;
            rx[u] = idx - sx[u] * R;
          }
          for (int m = 1; m < N; ++m) {
            int dg[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) dg[u] = sDig[sx[u] * NM + m - 1];
#pragma unroll
            for (int u = 0; u < 4; ++u) w[u] *= sA[offA[m] + dg[u] * R + rx[u]];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (base + u * kSmallThreads < S0 * R) sT0[base + u * kSmallThreads] = w[u];
        }
        __syncthreads();
      }
      if (n == 0) {
        // M^(0) = Z_(0) W on the matrix cores: 16-row tiles of mode 0 by the R
        // columns, the fibres s (the contraction) four per step; with fewer
        // row tiles than waves the fibres are split into KC chunks whose
        // partial tiles are then added in chunk order
        const int nt = (I0 + 15) >> 4;
        const int KC = nt >= kSmallWaves ? 1 : kSmallWaves / nt;
        const int chunk = ((S0 + KC - 1) / KC + 3) & ~3;
        for (int w = wave; w < nt * KC; w += kSmallWaves) {
          const int t = w % nt, kc = w / nt;
          const int sb = kc * chunk, se = sb + chunk < S0 ? sb + chunk : S0;
          const int i = t * 16 + lc;
          const int ic = i < I0 ? i : I0 - 1, cc = lc < R ? lc : R - 1;
          sd4 acc = {0.0, 0.0, 0.0, 0.0};
          // four steps per round, every operand load issued before the first
          // product (addresses clamped in range, masked entries zeroed after)
          for (int s0 = sb; s0 < se; s0 += 16) {
            double av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int sc = s0 + 4 * u + lj < S0 ? s0 + 4 * u + lj : S0 - 1;
              av[u] = (double)sZ[sc * I0p + ic];
              bv[u] = sT0[sc * R + cc];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const bool in = s0 + 4 * u + lj < se;
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64((in && i < I0) ? av[u] : 0.0,
                                                        (in && lc < R) ? bv[u] : 0.0, acc, 0, 0, 0);
            }
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = t * 16 + lj + 4 * v;   // result rows interleave as g + 4v
            if (lc < R && row < I0) {
              if (KC == 1) sM[row * R + lc] = acc[v];
              else sRed[(kc * nt + t) * 16 * R + (lj + 4 * v) * R + lc] = acc[v];
            }
          }
        }
        if (KC > 1) {
          __syncthreads();
          for (int idx = tid; idx < I0 * R; idx += kSmallThreads) {
            const int i = idx / R, c = idx - (idx / R) * R;
            const double* p = sRed + ((i >> 4) * 16 + (i & 15)) * R + c;
            sM[idx] = sum4(p, KC, nt * 16 * R);
          }
        }
      }
      if (n > 0 && N == 3) {
        // three-way tensors: the fibres with s_n = i are s = i st[n] + k st[m]
        // over the index k of the other mode m, so every (row, column) pair
        // sums its I_m terms itself, the loads of eight terms issued first;
        // each row starts at its own k = i mod I_m and wraps around, so that
        // the rows of one wave read from different banks
        const int m = 3 - n, Im = I[m], tsd = st[m] * R;
        for (int q = tid; q < I[n] * R; q += kSmallThreads) {
          const int i = q / R, r = q - (q / R) * R;
          const double* tp = sT0 + i * st[n] * R + r;
          const double* ap = sA + offA[m] + r;
          int k = i % Im;
          double a4[4] = {0.0, 0.0, 0.0, 0.0};
          int c = 0;
          for (; c + 7 < Im; c += 8) {
            double tv[8], av[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              tv[u] = tp[k * tsd];
              av[u] = ap[k * R];
              k = k + 1 == Im ? 0 : k + 1;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) a4[u & 3] += tv[u] * av[u];
          }
          for (; c < Im; ++c) {
            a4[0] += tp[k * tsd] * ap[k * R];
            k = k + 1 == Im ? 0 : k + 1;
          }
          sM[q] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
        }
      }
      // M^(n), n >= 1, other orders: (row, column) pairs, the contraction
      // split over G thread groups
      const int pairs = (n == 0 || N == 3) ? 0 : I[n] * R;
      const int G = pairs >= kSmallThreads ? 1 : kSmallThreads / (pairs > 0 ? pairs : 1);
      const int rest = S0 / I[n];
      for (int q0 = 0; q0 < pairs; q0 += kSmallThreads) {
        const int q = q0 + tid % (pairs < kSmallThreads ? pairs : kSmallThreads);
        const int g = pairs < kSmallThreads ? tid / pairs : 0;
        double acc = 0.0;
        const bool live = (pairs < kSmallThreads) ? (g < G) : (q < pairs);
        if (live) {
          const int i = q % I[n], r = q / I[n];
          double a4[4] = {0.0, 0.0, 0.0, 0.0};
          // four accumulators with static indices (a runtime index would
          // move the array out of registers)
          {
            const int32_t* pr = sPerm + (n - 1) * S0 + i * rest;
            auto term = [&](int k) {
              const int s = pr[k];
              double w = sT0[s * R + r];
              for (int m = 1; m < N; ++m)
                if (m != n) w *= sA[offA[m] + sDig[s * NM + m - 1] * R + r];
              return w;
            };
            int k = g;
            for (; k + 3 * G < rest; k += 4 * G)
#pragma unroll
              for (int u = 0; u < 4; ++u) a4[u] += term(k + u * G);
            for (; k < rest; k += G) a4[0] += term(k);
          }
          acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
        }
        if (pairs < kSmallThreads) {
          if (live) sRed[g * pairs + q] = acc;
          __syncthreads();
          if (tid < pairs) sM[(tid % I[n]) * R + tid / I[n]] = sum4(sRed + tid, G, pairs);
        } else if (q < pairs) {
          sM[(q % I[n]) * R + q / I[n]] = acc;
        }
      }
      __syncthreads();
      // Gauss-Seidel on the rows of A^(n), one thread per row
      gs_rows_any<kSmallThreads>(sA + offA[n], sM, sF + offA[n], sG, I[n], R, d.gs_iters);
      __syncthreads();
      gram(n);
      if (n == 0 && N > 1) {
        // stage-1 tiles of the updated A^(0) for the modes >= 1 of this sweep,
        // T0 = Z_(0)^T A^(0) on the matrix cores: 16 fibres by the R columns
        // per tile, mode 0 (the contraction) four entries per step
        const double* a0 = sA + offA[0];
        for (int s0 = wave * 16; s0 < S0; s0 += 16 * kSmallWaves) {
          const int s = s0 + lc;
          const T* zf = sZ + (s < S0 ? s : S0 - 1) * I0p;
          const int cc = lc < R ? lc : R - 1;
          sd4 acc = {0.0, 0.0, 0.0, 0.0};
          for (int k0 = 0; k0 < I0; k0 += 16) {
            double av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int kc = k0 + 4 * u + lj < I0 ? k0 + 4 * u + lj : I0 - 1;
              av[u] = (double)zf[kc];
              bv[u] = a0[kc * R + cc];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const bool in = k0 + 4 * u + lj < I0;
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64((in && s < S0) ? av[u] : 0.0,
                                                        (in && lc < R) ? bv[u] : 0.0, acc, 0, 0, 0);
            }
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int so = s0 + lj + 4 * v;
            if (lc < R && so < S0) sT0[so * R + lc] = acc[v];
          }
        }
      }
      __syncthreads();
    }
  }
  for (int m = 0; m < N; ++m)
    for (int idx = tid; idx < I[m] * R; idx += kSmallThreads) {
      const double v = sA[offA[m] + idx];
      d.A[m][idx] = v;
      if (d.A32[m]) d.A32[m][idx] = (float)v;
    }
}

size_t small_lds_bytes(const SmallDesc& d, bool fp32) {
  return (size_t)small_layout(d, fp32 ? 4 : 8).bytes;
}

bool small_eligible(const SmallDesc& d, bool fp32) {
  if (d.N < 2 || d.N > kMaxOrder || d.R < 1 || d.R > 16) return false;
  for (int m = 1; m < d.N; ++m)
    if (d.dims[m] > 65535) return false;   // digits are held as 16-bit values
  return small_lds_bytes(d, fp32) <= kSmallLdsBytes;
}

hipError_t relax_small_launch(const SmallDesc& d, bool fp32, hipStream_t st) {
  if (!small_eligible(d, fp32)) return hipErrorInvalidValue;
  const size_t lds = small_lds_bytes(d, fp32);
  const void* k = fp32 ? (const void*)relax_small_kernel<float> : (const void*)relax_small_kernel<double>;
  static bool attr_set[2] = {false, false};
  const int ki = fp32 ? 1 : 0;
  if (!attr_set[ki]) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallLdsBytes);
    if (e != hipSuccess) return e;
    attr_set[ki] = true;
  }
  SmallDesc dd = d;
  void* args[] = {&dd};
  return hipLaunchKernel(k, dim3(1), dim3(kSmallThreads), args, lds, st);
}

}  // namespace cpamg

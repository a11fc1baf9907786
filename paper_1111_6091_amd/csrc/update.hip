// Row-wise epilogues of the MTTKRP (R x R solves of Section 3 and 5.2), Gram
// matrices, normalization eq. (10), objectives eq. (2)/(30) and utilities.
#include <algorithm>

#include "internal.hpp"
#include "smallla.hpp"
#include "sweep.hpp"

namespace cpamg {

constexpr int EPI_ROWS = 4;
constexpr int LDP = kMaxRank + 1;   // padded LDS row stride (doubles)

int epi_rows_per_wg() { return EPI_ROWS; }

// Block-wide sum of one double per thread (256 threads); result valid in thread 0.
__device__ inline double block_sum(double v, double* sred) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sred[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) / 64;
    for (int w = 0; w < nw; ++w) s += sred[w];
  }
  __syncthreads();
  return s;
}

// Last-block detection: every thread publishes its writes; returns true in all
// threads of the block that arrives last.  The counter is reset by that block.
__device__ inline bool arrive_last(int32_t* counter, int nblk, int* s_flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const int prev = atomicAdd(counter, 1);
    *s_flag = (prev == nblk - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = *s_flag != 0;
  if (last) __threadfence();
  return last;
}

// Sum p[k * stride] for k = k0, k0 + step, ... < count in increasing k, with
// 8 independent loads in flight per round (the index clamped into range, no
// branch around a load); the additions stay in order, and the padding adds
// exact zeros.
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int k0, int count,
                                              int step, size_t stride) {
  constexpr int Q = 8;
  double s = 0.0;
  if (count <= 0) return s;
  for (int k = k0; k < count; k += Q * step) {
    double v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int kk = k + q * step;
      v[q] = p[(size_t)min(kk, count - 1) * stride];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) s += k + q * step < count ? v[q] : 0.0;
  }
  return s;
}

// Sum the MTTKRP partials of this block's rows in a fixed order.  The
// (row, column) pairs are spread over thread groups that each take every G-th
// split; group sums are then added in group order.
__device__ inline void reduce_partials(const EpiDesc& d, int64_t row0, int nrows, double* sM,
                                       double* sT) {
  const int R = d.R;
  const int pairs = nrows * R;
  const int G = pairs > 0 ? max(1, min(kThreads / pairs, 16)) : 1;
  const int tid = threadIdx.x;
  if (tid < pairs * G) {
    const int pr = tid % pairs, g = tid / pairs;
    const int row = pr / R, col = pr % R;
    sT[g * (EPI_ROWS * kMaxRank) + pr] =
        strided_sum(d.partial + (row0 + row) * R + col, g, d.nsplit, G, (size_t)d.In * R);
  }
  __syncthreads();
  if (tid < pairs) {
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += sT[g * (EPI_ROWS * kMaxRank) + tid];
    sM[(tid / R) * LDP + tid % R] = s;
  }
  __syncthreads();
}

// Gauss-Seidel on one row x Gamma = b (Gamma in G), r = 0..R-1 in order, warm
// start x0; lane j < R holds b_j and x_j.  Every lane forms the same sum
// t = sum_k x_k Gamma(k, r) from broadcasts, in increasing k.
__device__ inline double wave_gs(double b, double x, const double* G, int R, int iters, int lane) {
  for (int it = 0; it < iters; ++it) {
    for (int r = 0; r < R; ++r) {
      const double dg = G[r * R + r];
      if (dg == 0.0) continue;
      double t = 0.0;
      for (int k = 0; k < R; ++k) t += wave_bcast(x, k) * G[k * R + r];
      const double br = wave_bcast(b, r);
      const double xr = wave_bcast(x, r);
      const double v = (br - t + xr * dg) / dg;
      if (lane == r) x = v;
    }
  }
  return x;
}

// The same Gauss-Seidel iterations with every lane holding the whole row
// (uniform across the wave) and Gamma in registers: no broadcasts or LDS reads
// inside the iteration.  The equations are scaled by the reciprocal pivots
// once, c_r = b_r / Gamma_rr and h[k][r] = Gamma_kr / Gamma_rr, so that
// x_r <- c_r - sum_{k != r} x_k h[k][r]; a zero pivot (and every r >= R) gets
// c_r = 0, h[.][r] = 0 and a unit term that keeps x_r as it is.  RM >= R.
template <int RM>
__device__ inline double wave_gs_reg(double b, double x, const double* G, int R, int iters, int lane) {
  double xv[RM], c[RM], keep[RM], h[RM][RM];
#pragma unroll
  for (int r = 0; r < RM; ++r) {
    xv[r] = r < R ? wave_bcast(x, r) : 0.0;
    const double br = r < R ? wave_bcast(b, r) : 0.0;
    const double dg = r < R ? G[r * R + r] : 0.0;
    const bool piv = dg != 0.0;
    const double dinv = piv ? 1.0 / dg : 0.0;
    keep[r] = piv ? 0.0 : 1.0;
    c[r] = br * dinv;
#pragma unroll
    for (int k = 0; k < RM; ++k) h[k][r] = (k < R && r < R) ? G[k * R + r] * dinv : 0.0;
  }
  // static indices only.  Per iteration the terms of the previous iterate
  // (k > r) are formed side by side first; each new x_r then enters the
  // pending values of the later components (serial chain per component: one
  // product and subtraction)
  for (int it = 0; it < iters; ++it) {
    double t[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      double u = 0.0;
#pragma unroll
      for (int k = r + 1; k < RM; ++k) u += xv[k] * h[k][r];
      t[r] = fma(xv[r], keep[r], c[r] - u);
    }
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      xv[r] = t[r];
#pragma unroll
      for (int j = r + 1; j < RM; ++j) t[j] -= xv[r] * h[r][j];
    }
  }
  double out = 0.0;
#pragma unroll
  for (int r = 0; r < RM; ++r)
    if (lane == r) out = xv[r];
  return out;
}

__device__ inline double wave_gs_any(double b, double x, const double* G, int R, int iters, int lane) {
  switch (R) {
    case 1: case 2: return wave_gs_reg<2>(b, x, G, R, iters, lane);
    case 3: return wave_gs_reg<3>(b, x, G, R, iters, lane);
    case 4: return wave_gs_reg<4>(b, x, G, R, iters, lane);
    case 5: return wave_gs_reg<5>(b, x, G, R, iters, lane);
    case 6: return wave_gs_reg<6>(b, x, G, R, iters, lane);
    case 7: case 8: return wave_gs_reg<8>(b, x, G, R, iters, lane);
    default: return wave_gs(b, x, G, R, iters, lane);
  }
}

// One block of rows of a mode epilogue; blk / nblk: this block's index and the
// number of blocks of the epilogue (blk * EPI_ROWS is its first row).
__device__ __forceinline__ void epi_body(const EpiDesc& d, int blk, int nblk) {
  __shared__ double sG[kMaxRank * kMaxRank];
  __shared__ double sM[EPI_ROWS * LDP];
  __shared__ double sT[16 * EPI_ROWS * kMaxRank];
  __shared__ double sC[2 * kMaxRank];
  __shared__ double sred[8];
  __shared__ int s_flag;
  // batched solve: nothing left in this phase, or the problem is in the other phase
  if (d.st && (!d.st->active || d.st->phase != d.run_phase)) return;
  const int R = d.R;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = (int64_t)blk * EPI_ROWS;
  const int nrows = (int)std::min<int64_t>(EPI_ROWS, d.In - row0);
  int kind = 0;
  // Gamma^(n) prepared by the MTTKRP launch (inverse / pseudoinverse / Gamma,
  // then the column scale of M^(n) and sigma^(n), normalized coordinates):
  // loaded into registers here, stored to LDS after the partial sums, so that
  // both sets of loads are in flight together
  constexpr int PQ = (kMaxRank * kMaxRank + 2 * kMaxRank + kThreads - 1) / kThreads;
  double pv[PQ];
  if (d.op == EPI_UPDATE) {
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int idx = tid + q * kThreads;
      pv[q] = idx < R * R + 2 * R ? d.prep_out[idx] : 0.0;
    }
    kind = *d.kind;
  } else if (d.op != EPI_STORE_M) {
    hadamard_gamma(d.grams, d.N, d.n, R, sG);
  }
  reduce_partials(d, row0, nrows, sM, sT);
  if (d.op == EPI_UPDATE) {
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int idx = tid + q * kThreads;
      if (idx < R * R) sG[idx] = pv[q];
      else if (idx < R * R + 2 * R) sC[idx - R * R] = pv[q];
    }
    __syncthreads();
  }

  if (d.op == EPI_STORE_M) {
    for (int idx = tid; idx < nrows * R; idx += kThreads) {
      const int row = idx / R, col = idx % R;
      d.outbuf[(row0 + row) * R + col] = sM[row * LDP + col];
    }
    return;
  }

  if (d.op == EPI_H || d.op == EPI_GRAD) {
    double sq = 0.0;
    if (tid < nrows * R) {
      const int row = tid / R, j = tid % R;
      const double* a = d.A + (row0 + row) * R;
      double h = 0.0;
      for (int k = 0; k < R; ++k) h += a[k] * sG[k * R + j];
      h -= sM[row * LDP + j];
      if (d.op == EPI_H) d.outbuf[(row0 + row) * R + j] = h;
      sq = h * h;
    }
    if (d.op == EPI_H) return;
    const double tot = block_sum(sq, sred);
    if (tid == 0) d.scal_part[blk] = tot;
    if (arrive_last(d.counter, nblk, &s_flag)) {
      double acc = 0.0;
      for (int b = tid; b < nblk; b += kThreads) acc += d.scal_part[b];
      const double tot2 = block_sum(acc, sred);
      if (tid == 0) {
        *d.scalar_out = d.accumulate ? (*d.scalar_out + tot2) : tot2;
        atomicExch(d.counter, 0);
      }
    }
    return;
  }

  // ---- EPI_UPDATE: the block's rows in normalized coordinates -------------
  // Gamma is block-diagonal over the column groups, so one solve of all R
  // columns solves every group; frozen groups (batched solve) keep their rows.
  const int NG = d.groups > 1 ? d.groups : 1;
  const int Rg = R / NG;
  double ip = 0.0, x = 0.0;
  bool wr = false;
  int64_t orow = 0;   // output element (orow, oc) of this thread
  int oc = 0;
  if (kind != 2) {
    // kinds 0 and 1: row solve x Gamma = b with X (sG) from the bookkeeping:
    // kind 0, X = W = L^-1 for Gamma = L L^T, so x = (b W^T) W, i.e.
    // y_i = sum_j W_ij b_j, then x_c = sum_i y_i W_ic; kind 1, X is the
    // pseudoinverse, x_c = sum_k b_k X_kc.  Thread t < nrows R takes element
    // (t / R, t % R); b and y pass through LDS; sums in increasing index order
    double* sB = sT;
    double* sY = sT + EPI_ROWS * LDP;
    const int rl = tid / R, c = tid % R;
    const bool act = tid < nrows * R;
    double m = 0.0;
    if (act) {
      m = sC[c] * sM[rl * LDP + c];
      sB[rl * LDP + c] = m + (d.F ? d.F[(row0 + rl) * R + c] : 0.0);
    }
    __syncthreads();
    const double* v = sB;
    if (kind == 0) {
      if (act) {
        double y = 0.0;
#pragma unroll 4
        for (int j = 0; j < R; ++j) y = fma(sG[c * R + j], sB[rl * LDP + j], y);
        sY[rl * LDP + c] = y;
      }
      __syncthreads();
      v = sY;
    }
    if (act) {
#pragma unroll 4
      for (int k = 0; k < R; ++k) x = fma(v[rl * LDP + k], sG[k * R + c], x);
      wr = !(d.st && d.st->frozen[c / Rg]);
      if (wr) ip = x * m;
      orow = row0 + rl;
      oc = c;
    }
  } else if (wave < nrows) {
    // Gauss-Seidel: wave w solves row w, lane = column
    const int64_t row = row0 + wave;
    const double m = (lane < R) ? sC[lane] * sM[wave * LDP + lane] : 0.0;
    const double b = (lane < R) ? m + (d.F ? d.F[row * R + lane] : 0.0) : 0.0;
    const double x0 = (lane < R) ? sC[R + lane] * d.A[row * R + lane] : 0.0;
    x = wave_gs_any(b, x0, sG, R, d.gs_iters, lane);
    wr = lane < R && !(d.st && d.st->frozen[lane / Rg]);
    if (wr) ip = x * m;
    orow = row;
    oc = lane;
  }
  // the block sums (barriers) before the global stores, which a barrier would
  // wait for
  double ipb[kMaxGroups];
  if (d.want_obj)
    for (int g = 0; g < NG; ++g) ipb[g] = block_sum((wr && oc / Rg == g) ? ip : 0.0, sred);
  if (wr) {
    if (!isfinite(x)) atomicOr(d.flags, CP_FLAG_NONFINITE);
    d.A[orow * R + oc] = x;
    if (d.A32) d.A32[orow * R + oc] = (float)x;
  }
  if (d.want_obj && tid == 0)
    for (int g = 0; g < NG; ++g) d.scal_part[(size_t)blk * NG + g] = ipb[g];
}

__global__ __launch_bounds__(kThreads) void epi_kernel(EpiDesc d) {
  epi_body(d, blockIdx.x, gridDim.x);
}

// Batched epilogues: tile t runs block tiles[t].y of the epilogue descs[tiles[t].x].
__global__ __launch_bounds__(kThreads) void epi_batched_kernel(const EpiDesc* __restrict__ descs,
                                                               const int2* __restrict__ tiles) {
  const int2 t = tiles[blockIdx.x];
  const EpiDesc& d = descs[t.x];
  epi_body(d, t.y, (int)((d.In + EPI_ROWS - 1) / EPI_ROWS));
}

hipError_t epi_batched_launch(const EpiDesc* descs, const int2* tiles, int ntiles, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(epi_batched_kernel, dim3(ntiles), dim3(kThreads), 0, st, descs, tiles);
  return hipGetLastError();
}

hipError_t epi_launch(const EpiDesc& d, hipStream_t st) {
  const unsigned nwg = (unsigned)((d.In + EPI_ROWS - 1) / EPI_ROWS);
  hipLaunchKernelGGL(epi_kernel, dim3(nwg), dim3(kThreads), 0, st, d);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void finalize_kernel(PrepArgs a) {
  extern __shared__ double dsmem[];
  sweep_prep<16>(a, dsmem, true);
}

hipError_t finalize_launch(const PrepArgs& a0, hipStream_t st) {
  PrepArgs a = a0;
  a.lds = prep_smem_doubles(a.N, a.R);
  const size_t bytes = sizeof(double) * a.lds;
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kThreads), bytes, st, a);
  return hipGetLastError();
}

// Batched: workgroup j finalizes problem plist[j] (pas[plist[j]]); smem_doubles
// covers the largest problem.
__global__ __launch_bounds__(kThreads) void finalize_batched_kernel(const PrepArgs* __restrict__ pas,
                                                                    const int32_t* __restrict__ plist) {
  extern __shared__ double dsmem[];
  sweep_prep<16>(pas[plist[blockIdx.x]], dsmem, true);
}

hipError_t finalize_batched_launch(const PrepArgs* pas, const int32_t* plist, int count,
                                   int smem_doubles, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_batched_kernel, dim3(count), dim3(kThreads),
                     sizeof(double) * (size_t)smem_doubles, st, pas, plist);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Grams of every mode (one workgroup per mode), optional FP32 shadow refresh.
struct GramArgs {
  double* A[kMaxOrder];
  float* A32[kMaxOrder];
  int64_t dims[kMaxOrder];
};

typedef double gd4 __attribute__((ext_vector_type(4)));

// R <= 16: U = A^T A on the matrix cores, as products of the 16-column row
// tile with itself (v_mfma_f64_16x16x4f64), four rows per step with the loads
// of a step issued first; the four waves take interleaved 16-row blocks and
// their tiles are added in wave order.
__device__ __forceinline__ void gram_body_mfma(const double* __restrict__ A, float* A32, int64_t I,
                                               int R, double* gram_out, double* sigma_out) {
  __shared__ double part[(kThreads / 64) * 256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lc = lane & 15, lj = lane >> 4;
  const int RR = R * R;
  const int rc = lc < R ? lc : R - 1;
  gd4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i0 = (int64_t)wave * 16; i0 < I; i0 += 16 * (kThreads / 64)) {
    double av[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t row = i0 + 4 * u + lj;
      av[u] = A[(row < I ? row : I - 1) * R + rc];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double v = (i0 + 4 * u + lj < I && lc < R) ? av[u] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = lj + 4 * v;   // result rows interleave as g + 4v
    if (row < R && lc < R) part[wave * RR + row * R + lc] = acc[v];
  }
  if (A32)
    for (int64_t idx = tid; idx < I * R; idx += kThreads) A32[idx] = (float)A[idx];
  __syncthreads();
  if (tid < RR) gram_out[tid] = (part[tid] + part[RR + tid]) + (part[2 * RR + tid] + part[3 * RR + tid]);
  if (sigma_out && tid < R) sigma_out[tid] = 1.0;
}

// Gram U = A^T A of one I x R factor into gram_out (R x R); refreshes the FP32
// shadow when A32 is set and resets the column scales when sigma_out is set.
__device__ __forceinline__ void gram_body(const double* __restrict__ A, float* A32, int64_t I, int R,
                                          double* gram_out, double* sigma_out) {
  if (R <= 16) {
    gram_body_mfma(A, A32, I, R, gram_out, sigma_out);
    return;
  }
  __shared__ double tile[64 * LDP];
  double acc[4] = {0, 0, 0, 0};
  for (int64_t i0 = 0; i0 < I; i0 += 64) {
    const int rows = (int)std::min<int64_t>(64, I - i0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < rows * R; idx += kThreads) {
      const double v = A[i0 * R + idx];
      tile[(idx / R) * LDP + idx % R] = v;
      if (A32) A32[i0 * R + idx] = (float)v;
    }
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      const int idx = threadIdx.x + q * kThreads;
      if (idx < R * R) {
        const int a = idx / R, b = idx % R;
        double s = acc[q];
        for (int row = 0; row < rows; ++row) s += tile[row * LDP + a] * tile[row * LDP + b];
        acc[q] = s;
      }
    }
  }
  for (int q = 0; q < 4; ++q) {
    const int idx = threadIdx.x + q * kThreads;
    if (idx < R * R) gram_out[idx] = acc[q];
  }
  if (sigma_out && threadIdx.x < R) sigma_out[threadIdx.x] = 1.0;
}

__global__ __launch_bounds__(kThreads) void gram_kernel(GramArgs g, int R, double* grams,
                                                        double* sigma) {
  const int m = blockIdx.x;
  gram_body(g.A[m], g.A32[m], g.dims[m], R, grams + (size_t)m * R * R,
            sigma ? sigma + (size_t)m * R : nullptr);
}

// Batched: workgroup j computes mode j % N of problem plist[j / N]
// (jobs[problem * N + mode]); problems with nothing left in the current phase
// are skipped.
__global__ __launch_bounds__(kThreads) void gram_batched_kernel(const GramJob* __restrict__ jobs,
                                                                const int32_t* __restrict__ plist,
                                                                int N) {
  const GramJob& j = jobs[(size_t)plist[blockIdx.x / N] * N + blockIdx.x % N];
  if (j.st && !j.st->active) return;
  gram_body(j.A, j.A32, j.I, j.R, j.gram, j.sigma);
}

hipError_t gram_batched_launch(const GramJob* jobs, const int32_t* plist, int count, int N,
                               hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(gram_batched_kernel, dim3(count * N), dim3(kThreads), 0, st, jobs, plist, N);
  return hipGetLastError();
}

hipError_t gram_launch(double* const* A, float* const* A32, const int64_t* dims, int N, int R,
                       double* grams, hipStream_t st, double* sigma) {
  GramArgs g{};
  for (int m = 0; m < N; ++m) {
    g.A[m] = A[m];
    g.A32[m] = A32 ? A32[m] : nullptr;
    g.dims[m] = dims[m];
  }
  hipLaunchKernelGGL(gram_kernel, dim3(N), dim3(kThreads), 0, st, g, R, grams, sigma);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exact residual 1/2 ||Z - [[A]]||^2: one pass over Z; each block takes a range
// of mode-0 fibres.  It forms the weights W_f(r) = prod_{m>=1} A^(m)(f_m, r) of
// all its fibres at once (LDS), stages A^(0) in LDS when it fits, and then each
// thread walks its rows i0 across the block's fibres, four fibres at a time
// with their tensor loads issued first.
struct ResArgs {
  const double* A[kMaxOrder];
  int64_t dims[kMaxOrder];
};

constexpr int kResA0 = 4096;   // doubles of A^(0) staged in LDS at most
constexpr int kResW = 2048;    // doubles of fibre weights per block

template <bool STAGED>
__device__ __forceinline__ double residual_rows(const double* __restrict__ z, const double* a0,
                                                const double* sW, int64_t I0, int R, int64_t fb,
                                                int nf) {
  double acc = 0.0;
  for (int64_t i0 = threadIdx.x; i0 < I0; i0 += kThreads) {
    const double* arow = a0 + i0 * R;
    int fl = 0;
    for (; fl + 3 < nf; fl += 4) {
      double zv[4], m4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int u = 0; u < 4; ++u) zv[u] = z[(fb + fl + u) * I0 + i0];
      for (int r = 0; r < R; ++r) {
        const double a = arow[r];
#pragma unroll
        for (int u = 0; u < 4; ++u) m4[u] += a * sW[(fl + u) * R + r];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double df = zv[u] - m4[u];
        acc += df * df;
      }
    }
    for (; fl < nf; ++fl) {
      const double zv = z[(fb + fl) * I0 + i0];
      double mdl = 0.0;
      for (int r = 0; r < R; ++r) mdl += arow[r] * sW[fl * R + r];
      const double df = zv - mdl;
      acc += df * df;
    }
  }
  return acc;
}

__global__ __launch_bounds__(kThreads) void residual_kernel(const double* __restrict__ z,
                                                            ResArgs ra, int N, int R,
                                                            int64_t fibres, int64_t fpb,
                                                            double* part, int32_t* counter,
                                                            double* f) {
  __shared__ double sA0[kResA0];
  __shared__ double sW[kResW];
  __shared__ double sred[8];
  __shared__ int s_flag;
  const int64_t I0 = ra.dims[0];
  const int64_t fb0 = (int64_t)blockIdx.x * fpb;
  const int64_t fe = std::min<int64_t>(fibres, fb0 + fpb);
  const int fcap = kResW / R;   // fibres whose weights fit in sW at once
  const bool staged = I0 * R <= kResA0;
  if (staged)
    for (int idx = threadIdx.x; idx < I0 * R; idx += kThreads) sA0[idx] = ra.A[0][idx];
  double acc = 0.0;
  for (int64_t fb = fb0; fb < fe; fb += fcap) {
    const int nf = (int)std::min<int64_t>(fcap, fe - fb);
    if (fb != fb0) __syncthreads();   // the previous fibres' weights are consumed
    for (int idx = threadIdx.x; idx < nf * R; idx += kThreads) {
      const int fl = idx / R, r = idx - (idx / R) * R;
      int64_t q = fb + fl;
      double w = 1.0;
      for (int m = 1; m < N; ++m) {
        const int64_t im = q % ra.dims[m];
        q /= ra.dims[m];
        w *= ra.A[m][im * R + r];
      }
      sW[idx] = w;
    }
    __syncthreads();
    acc += staged ? residual_rows<true>(z, sA0, sW, I0, R, fb, nf)
                  : residual_rows<false>(z, ra.A[0], sW, I0, R, fb, nf);
  }
  const double tot = block_sum(acc, sred);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
  if (arrive_last(counter, (int)gridDim.x, &s_flag)) {
    // the last block adds the block sums, every thread a strided share
    double s = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kThreads) s += part[b];
    const double all = block_sum(s, sred);
    if (threadIdx.x == 0) {
      *f = 0.5 * all;
      atomicExch(counter, 0);
    }
  }
}

hipError_t residual_launch(const double* z, const int64_t* dims, int N, int R,
                           const double* const* A, double* part, int32_t* counter, double* f,
                           hipStream_t st) {
  ResArgs ra{};
  int64_t fibres = 1;
  for (int m = 0; m < N; ++m) {
    ra.A[m] = A[m];
    ra.dims[m] = dims[m];
    if (m >= 1) fibres *= dims[m];
  }
  // about 8k entries per block (whose weights sW holds at once), at most 2048
  // blocks (a block then walks its fibres in groups that sW holds)
  int64_t fpb = std::max<int64_t>(1, 8192 / std::max<int64_t>(1, dims[0]));
  fpb = std::min<int64_t>(fpb, kResW / R);
  int64_t nb = (fibres + fpb - 1) / fpb;
  if (nb > 2048) {
    fpb = (fibres + 2047) / 2048;
    nb = (fibres + fpb - 1) / fpb;
  }
  hipLaunchKernelGGL(residual_kernel, dim3((unsigned)nb), dim3(kThreads), 0, st, z, ra, N, R,
                     fibres, fpb, part, counter, f);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void dot_kernel(const double* __restrict__ a,
                                                       const double* __restrict__ b,
                                                       int64_t count, double* part,
                                                       int32_t* counter, double* out) {
  __shared__ double sred[8];
  __shared__ int s_flag;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * kThreads)
    acc += a[i] * (b ? b[i] : a[i]);
  const double tot = block_sum(acc, sred);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
  if (arrive_last(counter, (int)gridDim.x, &s_flag)) {
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int k = 0; k < (int)gridDim.x; ++k) s += part[k];
      *out = s;
      atomicExch(counter, 0);
    }
  }
}

static unsigned dot_blocks(int64_t count) {
  int64_t nb = (count + kThreads * 8 - 1) / (kThreads * 8);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(nb, 1024));
}

hipError_t norm2_launch(const double* z, int64_t count, double* part, int32_t* counter,
                        double* out, hipStream_t st) {
  hipLaunchKernelGGL(dot_kernel, dim3(dot_blocks(count)), dim3(kThreads), 0, st, z,
                     (const double*)nullptr, count, part, counter, out);
  return hipGetLastError();
}

hipError_t inner_launch(const double* A, const double* M, int64_t count, double* part,
                        int32_t* counter, double* out, hipStream_t st) {
  hipLaunchKernelGGL(dot_kernel, dim3(dot_blocks(count)), dim3(kThreads), 0, st, A, M, count,
                     part, counter, out);
  return hipGetLastError();
}

__global__ void fused_f_kernel(const double* grams, int N, int R, const double* inner,
                               const double* norm2, double* f) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double nrm = 0.0;
    for (int idx = 0; idx < R * R; ++idx) {
      double h = 1.0;
      for (int m = 0; m < N; ++m) h *= grams[(size_t)m * R * R + idx];
      nrm += h;
    }
    *f = 0.5 * (*norm2 - 2.0 * (*inner) + nrm);
  }
}

hipError_t fused_f_launch(const double* grams, int N, int R, const double* inner,
                          const double* norm2, double* f, hipStream_t st) {
  hipLaunchKernelGGL(fused_f_kernel, dim3(1), dim3(64), 0, st, grams, N, R, inner, norm2, f);
  return hipGetLastError();
}

__global__ void finish_g_kernel(const double* acc, const double* norm2, double* g) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *g = sqrt(*acc) / sqrt(*norm2);
}

hipError_t finish_g_launch(const double* acc, const double* norm2, double* g, hipStream_t st) {
  hipLaunchKernelGGL(finish_g_kernel, dim3(1), dim3(64), 0, st, acc, norm2, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void cast_kernel(const double* __restrict__ s, float* __restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = (float)s[i];
}

hipError_t cast_launch(const double* src, float* dst, int64_t count, hipStream_t st) {
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 1023) / 1024, 4096));
  hipLaunchKernelGGL(cast_kernel, dim3(nb), dim3(kThreads), 0, st, src, dst, count);
  return hipGetLastError();
}

__global__ void fill_kernel(double* d, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = v;
}

hipError_t fill_launch(double* dst, double v, int64_t count, hipStream_t st) {
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 1023) / 1024, 4096));
  hipLaunchKernelGGL(fill_kernel, dim3(nb), dim3(kThreads), 0, st, dst, v, count);
  return hipGetLastError();
}

__global__ void copy_kernel(const double* __restrict__ s, double* __restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

hipError_t copy_launch(const double* src, double* dst, int64_t count, hipStream_t st) {
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 1023) / 1024, 4096));
  hipLaunchKernelGGL(copy_kernel, dim3(nb), dim3(kThreads), 0, st, src, dst, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stable sort of the components by decreasing lambda_r (one workgroup).
__global__ __launch_bounds__(kThreads) void sort_kernel(GramArgs g, int N, int R) {
  __shared__ double lam[kMaxRank];
  __shared__ int perm[kMaxRank];
  __shared__ double rowbuf[kThreads / kMaxRank + 1][kMaxRank];
  if (threadIdx.x < R) {
    const int r = threadIdx.x;
    double prod = 1.0;
    for (int m = 0; m < N; ++m) {
      double s = 0.0;
      for (int64_t i = 0; i < g.dims[m]; ++i) {
        const double v = g.A[m][i * R + r];
        s += v * v;
      }
      prod *= sqrt(s);
    }
    lam[r] = pow(prod, 1.0 / N);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int r = 0; r < R; ++r) perm[r] = r;
    for (int i = 1; i < R; ++i) {   // insertion sort: stable, decreasing lambda
      const int p = perm[i];
      int j = i - 1;
      while (j >= 0 && lam[perm[j]] < lam[p]) {
        perm[j + 1] = perm[j];
        --j;
      }
      perm[j + 1] = p;
    }
  }
  __syncthreads();
  // permute columns row by row; each thread owns one row at a time
  for (int m = 0; m < N; ++m) {
    for (int64_t i = threadIdx.x; i < g.dims[m]; i += kThreads) {
      double tmp[kMaxRank];
      for (int r = 0; r < R; ++r) tmp[r] = g.A[m][i * R + perm[r]];
      for (int r = 0; r < R; ++r) {
        g.A[m][i * R + r] = tmp[r];
        if (g.A32[m]) g.A32[m][i * R + r] = (float)tmp[r];
      }
    }
  }
  (void)rowbuf;
}

hipError_t sort_launch(double* const* A, float* const* A32, const int64_t* dims, int N, int R,
                       double* scratch, hipStream_t st) {
  (void)scratch;
  GramArgs g{};
  for (int m = 0; m < N; ++m) {
    g.A[m] = A[m];
    g.A32[m] = A32 ? A32[m] : nullptr;
    g.dims[m] = dims[m];
  }
  hipLaunchKernelGGL(sort_kernel, dim3(1), dim3(kThreads), 0, st, g, N, R);
  return hipGetLastError();
}

}  // namespace cpamg

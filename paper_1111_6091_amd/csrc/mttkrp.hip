// Dense MTTKRP  M^(n) = Z_(n) Phi^(n)  (eq. (6)-(7)) on gfx950.
//
// Stage 1 is a GEMM on the matrix cores that contracts one mode of Z with its
// factor: v_mfma_f64_16x16x4f64 (FP64) or v_mfma_f32_16x16x4f32 (mixed form,
// FP32 accumulation).  Stage 2 is a Hadamard-reduce of the GEMM tile with the
// factors of the remaining modes, in FP64.  The Khatri-Rao matrix is never
// formed.  The tensor is streamed once per call with 16- or 32-byte loads per
// lane; the GEMM operand layout makes every group of 16 lanes read 64
// consecutive entries (kind 1) or every 4 lanes one 16-entry fibre segment
// (kinds 2/3).
//
// MFMA 16x16x4 operand layout (one 64-lane wave): lane l supplies
//   A[m = l%16][k = l/16], B[k = l/16][n = l%16], and receives
//   D[m = mfma_row<T>(l/16, v)][n = l%16], v = 0..3 (see internal.hpp).
#include "internal.hpp"
#include "smallla.hpp"
#include "sweep.hpp"

namespace cpamg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Vec4;
template <> struct Vec4<double> { typedef d4 type; };
template <> struct Vec4<float> { typedef f4 type; };

__device__ __forceinline__ d4 mma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Load 4 consecutive entries p[0..3]; entries at index >= nvalid read as 0.
template <typename T, bool VEC>
__device__ __forceinline__ typename Vec4<T>::type load4(const T* __restrict__ p, int nvalid) {
  typedef typename Vec4<T>::type V;
  V v;
  if (VEC) {
    if (nvalid >= 4) {
      v = *reinterpret_cast<const V*>(p);
    } else {
      v = V{0, 0, 0, 0};
    }
  } else {
    v[0] = nvalid > 0 ? p[0] : T(0);
    v[1] = nvalid > 1 ? p[1] : T(0);
    v[2] = nvalid > 2 ? p[2] : T(0);
    v[3] = nvalid > 3 ? p[3] : T(0);
  }
  return v;
}

// 32 bytes per lane: VW = 4 doubles or 8 floats, as one or two 4-wide loads.
template <typename T> struct VW_ { static constexpr int value = 32 / sizeof(T); };

template <typename T, bool VEC>
__device__ __forceinline__ void loadw(const T* __restrict__ p, int nvalid, T (&out)[VW_<T>::value]) {
  constexpr int VW = VW_<T>::value;
#pragma unroll
  for (int q = 0; q < VW / 4; ++q) {
    const int nv = nvalid - 4 * q;
    const typename Vec4<T>::type v = load4<T, VEC>(p + 4 * q, nv < 0 ? 0 : (nv > 4 ? 4 : nv));
#pragma unroll
    for (int e = 0; e < 4; ++e) out[4 * q + e] = v[e];
  }
}

// Product of the stripe-mode factors at stripe s, column col (skip mode `skip`).
__device__ __forceinline__ double stripe_weight(const MttkrpDesc& d, int64_t s, int col, int skip) {
  if (col >= d.R) return 0.0;
  double w = 1.0;
  for (int j = 0; j < d.ns; ++j) {
    const int m = j + 2;
    const int64_t sj = (s / d.sst[j]) % d.sext[j];
    if (m != skip) w *= d.a64[m][sj * d.R + col];
  }
  return w;
}

constexpr int kSmem = kPrepSmem;   // doubles of LDS per workgroup (40 KB)
static_assert(kSmem >= 4096, "reduction buffers need 4096 doubles");

// Workgroup 0 of a launch with prep set does the sweep bookkeeping for the
// update that follows (sweep.hpp), concurrently with the streaming workgroups;
// it is dispatched first, so it is resident from the start.
__device__ __forceinline__ bool prep_block(const MttkrpDesc& d, double* smem) {
  if (!d.prep || blockIdx.x != 0) return false;
  sweep_prep(d.pa, smem, false);
  return true;
}

// ---------------------------------------------------------------------------
// kind 1: output mode 0.  Each lane loads VW consecutive rows i0 at one i1;
// sub-tile a holds rows i0 = grp*16*VW + VW*m + a (m = GEMM row).  Contraction
// over i1 on the matrix cores, Hadamard weight per stripe in FP64.
// ---------------------------------------------------------------------------
template <typename T, int NT, bool VEC>
__global__ __launch_bounds__(kThreads) void mttkrp_kind1(MttkrpDesc d) {
  typedef typename Vec4<T>::type V;
  constexpr int VW = VW_<T>::value;
  constexpr int PANEL = 16 * VW;
  __shared__ double smem[kSmem];
  if (prep_block(d, smem)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g4 = lane >> 4;
  const int bid = blockIdx.x - d.prep;
  const int grp = bid % d.ngroups;
  const int split = bid / d.ngroups;
  const T* __restrict__ z = reinterpret_cast<const T*>(d.z);
  const T* __restrict__ ak = reinterpret_cast<const T*>(d.ak);
  const int R = d.R;
  const int64_t I0 = d.I0, I1 = d.I1;
  const int64_t i0b = (int64_t)grp * PANEL + VW * r;   // first of this lane's VW rows
  const int64_t left = I0 - i0b;
  const int nrow = left <= 0 ? 0 : (left >= VW ? VW : (int)left);

  double acc[VW][NT][4];
#pragma unroll
  for (int a = 0; a < VW; ++a)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][t][v] = 0.0;

  const int64_t ubeg = (int64_t)split * d.chunk;
  const int64_t uend = min(d.units, ubeg + d.chunk);
  for (int64_t u = ubeg + wave; u < uend; u += 4) {
    const int64_t s = u / d.ksplit;
    const int kp = (int)(u % d.ksplit);
    const int64_t kbeg = (int64_t)kp * d.kchunk;
    const int64_t kend = min(I1, kbeg + d.kchunk);
    double w[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) w[t] = stripe_weight(d, s, t * 16 + r, -1);
    V D[VW][NT];
#pragma unroll
    for (int a = 0; a < VW; ++a)
#pragma unroll
      for (int t = 0; t < NT; ++t) D[a][t] = V{0, 0, 0, 0};
    const T* __restrict__ zs = z + (size_t)s * I0 * I1 + i0b;
    for (int64_t k0 = kbeg; k0 < kend; k0 += 16) {
      T zv[4][VW];
      T b[4][NT];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i1 = k0 + 4 * g4 + e;
        const bool ok = i1 < kend;
        loadw<T, VEC>(zs + (ok ? i1 : 0) * I0, ok ? nrow : 0, zv[e]);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int col = t * 16 + r;
          b[e][t] = (ok && col < R) ? ak[i1 * R + col] : T(0);
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int a = 0; a < VW; ++a)
#pragma unroll
          for (int t = 0; t < NT; ++t) D[a][t] = mma(zv[e][a], b[e][t], D[a][t]);
    }
    // Hadamard-reduce with the stripe weight (FP64)
#pragma unroll
    for (int a = 0; a < VW; ++a)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[a][t][v] += (double)D[a][t][v] * w[t];
  }
  // deterministic cross-wave reduction through LDS, 4 sub-tiles x 16 columns at
  // a time: GEMM row m of sub-tile a holds i0 = grp*PANEL + VW*m + a
#pragma unroll
  for (int a0 = 0; a0 < VW; a0 += 4)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      __syncthreads();
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          smem[(wave * 64 + mfma_row<T>(g4, v) * 4 + a) * 16 + r] = acc[a0 + a][t][v];
      __syncthreads();
      for (int idx = threadIdx.x; idx < 64 * 16; idx += kThreads) {
        const int q = idx / 16, c = idx % 16;   // q = 4*m + a
        const int m = q >> 2, a = q & 3;
        const int64_t i0 = (int64_t)grp * PANEL + VW * m + a0 + a;
        const int col = t * 16 + c;
        if (col < R && i0 < I0) {
          const double sum = smem[idx] + smem[1024 + idx] + smem[2048 + idx] + smem[3072 + idx];
          d.out[((size_t)split * d.In + i0) * R + col] = sum;
        }
      }
    }
}

// ---------------------------------------------------------------------------
// kinds 2 and 3: GEMM rows = i1 (16*TW per wave), contraction over i0 with VW
// consecutive i0 per lane.  kind 2 (n == 1): rows are the outputs; kind 3
// (n >= 2): rows are reduced with A^(1)(i1, r) into output s_n.
// ---------------------------------------------------------------------------
template <typename T, int NT, int TW, bool KIND3, bool VEC>
__global__ __launch_bounds__(kThreads) void mttkrp_kind23(MttkrpDesc d) {
  typedef typename Vec4<T>::type V;
  constexpr int VW = VW_<T>::value;
  constexpr int KC = 4 * VW;   // contraction chunk per step of the loop
  constexpr int ROWS = 16 * TW;
  __shared__ double smem[kSmem];
  if (prep_block(d, smem)) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, g4 = lane >> 4;
  const int bid = blockIdx.x - d.prep;
  const int grp = bid % d.ngroups;
  const int split = bid / d.ngroups;
  const T* __restrict__ z = reinterpret_cast<const T*>(d.z);
  const T* __restrict__ ak = reinterpret_cast<const T*>(d.ak);
  const int R = d.R;
  const int64_t I0 = d.I0, I1 = d.I1;

  // kind 2: acc[tw][t][v] holds row grp*ROWS + tw*16 + mfma_row<T>(g4, v)
  // kind 3: acc[0][t][0] holds the running sum for column t*16 + r
  double acc[TW][NT][4];
#pragma unroll
  for (int a = 0; a < TW; ++a)
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[a][t][v] = 0.0;

  const int64_t ubeg = (int64_t)split * d.chunk;
  const int64_t uend = min(d.units, ubeg + d.chunk);
  const int jn = d.n - 2;
  const int64_t stride_n = KIND3 ? d.sst[jn] : 1;
  for (int64_t u = ubeg + wave; u < uend; u += 4) {
    const int kp = (int)(u % d.ksplit);
    const int64_t uu = u / d.ksplit;
    int64_t s, rowbase;
    if (KIND3) {
      const int64_t g = uu % d.rgroups;
      int64_t q = uu / d.rgroups;
      rowbase = g * ROWS;
      // stripe from output value grp (mode n) and rest index q (other stripe modes)
      s = (int64_t)grp * stride_n;
      for (int j = 0; j < d.ns; ++j) {
        if (j == jn) continue;
        const int64_t sj = q % d.sext[j];
        q /= d.sext[j];
        s += sj * d.sst[j];
      }
    } else {
      s = uu;
      rowbase = (int64_t)grp * ROWS;
    }
    const int64_t kbeg = (int64_t)kp * d.kchunk;
    const int64_t kend = min(I0, kbeg + d.kchunk);
    double w[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) w[t] = stripe_weight(d, s, t * 16 + r, KIND3 ? d.n : -1);
    V D[TW][NT];
#pragma unroll
    for (int a = 0; a < TW; ++a)
#pragma unroll
      for (int t = 0; t < NT; ++t) D[a][t] = V{0, 0, 0, 0};
    const T* __restrict__ zs = z + (size_t)s * I0 * I1;
    bool rowok[TW];
#pragma unroll
    for (int a = 0; a < TW; ++a) rowok[a] = (rowbase + a * 16 + r) < I1;
    for (int64_t k0 = kbeg; k0 < kend; k0 += KC) {
      const int64_t kl = k0 + VW * g4;
      const int64_t nk = kend - kl;
      const int nval = nk >= VW ? VW : (nk > 0 ? (int)nk : 0);
      T zv[TW][VW];
#pragma unroll
      for (int a = 0; a < TW; ++a) {
        const int64_t i1 = rowbase + a * 16 + r;
        loadw<T, VEC>(zs + (rowok[a] ? i1 : 0) * I0 + (nval ? kl : 0), rowok[a] ? nval : 0, zv[a]);
      }
      T b[VW][NT];
#pragma unroll
      for (int e = 0; e < VW; ++e)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int col = t * 16 + r;
          b[e][t] = (e < nval && col < R) ? ak[(kl + e) * R + col] : T(0);
        }
#pragma unroll
      for (int e = 0; e < VW; ++e)
#pragma unroll
        for (int a = 0; a < TW; ++a)
#pragma unroll
          for (int t = 0; t < NT; ++t) D[a][t] = mma(zv[a][e], b[e][t], D[a][t]);
    }
    // Hadamard-reduce (FP64)
    if (KIND3) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int col = t * 16 + r;
        double part = 0.0;
#pragma unroll
        for (int a = 0; a < TW; ++a)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t i1 = rowbase + a * 16 + mfma_row<T>(g4, v);
            const double a1 = (i1 < I1 && col < R) ? d.a64[1][i1 * R + col] : 0.0;
            part += (double)D[a][t][v] * a1;
          }
        acc[0][t][0] += part * w[t];
      }
    } else {
#pragma unroll
      for (int a = 0; a < TW; ++a)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[a][t][v] += (double)D[a][t][v] * w[t];
    }
  }
  if (KIND3) {
    // reduce over the 4 lane groups (rows), then over waves in fixed order
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      double x = acc[0][t][0];
      x += __shfl_xor(x, 16);
      x += __shfl_xor(x, 32);
      if (g4 == 0) smem[wave * 16 * NT + t * 16 + r] = x;
    }
    __syncthreads();
    if (threadIdx.x < 16 * NT) {
      const int col = threadIdx.x;
      if (col < R) {
        const double sum = smem[col] + smem[16 * NT + col] + smem[32 * NT + col] + smem[48 * NT + col];
        d.out[((size_t)split * d.In + grp) * R + col] = sum;
      }
    }
  } else {
    static_assert(4 * ROWS * 16 * NT <= kSmem, "reduction buffer");
#pragma unroll
    for (int a = 0; a < TW; ++a)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          smem[(wave * ROWS + a * 16 + mfma_row<T>(g4, v)) * (16 * NT) + t * 16 + r] = acc[a][t][v];
    __syncthreads();
    for (int idx = threadIdx.x; idx < ROWS * 16 * NT; idx += kThreads) {
      const int row = idx / (16 * NT), col = idx % (16 * NT);
      const int64_t i1 = (int64_t)grp * ROWS + row;
      if (col < R && i1 < I1) {
        const int st = ROWS * 16 * NT;
        const double sum = smem[idx] + smem[st + idx] + smem[2 * st + idx] + smem[3 * st + idx];
        d.out[((size_t)split * d.In + i1) * R + col] = sum;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host side: planning and dispatch
// ---------------------------------------------------------------------------
static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

MttkrpPlan mttkrp_plan(int N, const int64_t* dims, int n, int R, int target_wgs, bool fp32) {
  MttkrpPlan p{};
  const int64_t I0 = dims[0], I1 = dims[1];
  int64_t S = 1;
  for (int m = 2; m < N; ++m) S *= dims[m];
  const int64_t vw = fp32 ? 8 : 4;   // elements per 32-byte lane load
  p.nt = R <= 16 ? 1 : 2;
  p.tw = 2;
  const int64_t rows = 16 * p.tw;
  int64_t base_units, K, kgran;
  if (n == 0) {
    p.kind = 1;
    p.ngroups = (int32_t)ceil_div(I0, 16 * vw);
    base_units = S;
    K = I1;
    kgran = 16;
  } else if (n == 1) {
    p.kind = 2;
    p.ngroups = (int32_t)ceil_div(I1, rows);
    base_units = S;
    K = I0;
    kgran = 4 * vw;
  } else {
    p.kind = 3;
    p.ngroups = (int32_t)dims[n];
    p.rgroups = (int32_t)ceil_div(I1, rows);
    base_units = p.rgroups * (S / dims[n]);
    K = I0;
    kgran = 4 * vw;
  }
  // split the contraction when there are too few (group, unit) pairs for the chip
  const int64_t want_units = (int64_t)target_wgs * 4;
  int64_t ks = 1;
  const int64_t kchunks = ceil_div(K, kgran);
  if ((int64_t)p.ngroups * base_units < want_units)
    ks = std::min<int64_t>(kchunks, ceil_div(want_units, (int64_t)p.ngroups * base_units));
  if (ks < 1) ks = 1;
  const int64_t kchunk = ceil_div(kchunks, ks) * kgran;
  ks = ceil_div(K, kchunk);
  p.ksplit = (int32_t)ks;
  p.kchunk = (int32_t)kchunk;
  p.units = base_units * ks;
  int64_t nsplit = std::max<int64_t>(1, target_wgs / p.ngroups);
  nsplit = std::min<int64_t>(nsplit, std::max<int64_t>(1, ceil_div(p.units, 4)));
  p.chunk = ceil_div(p.units, nsplit);
  p.nsplit = (int32_t)ceil_div(p.units, p.chunk);
  p.partial_doubles = (size_t)p.nsplit * dims[n] * R;
  return p;
}

template <typename T, int NT>
static hipError_t launch_typed(const MttkrpPlan& p, const MttkrpDesc& d, bool vec,
                               hipStream_t st) {
  dim3 grid((unsigned)((int64_t)p.ngroups * p.nsplit + (d.prep ? 1 : 0))), block(kThreads);
  if (p.kind == 1) {
    if (vec) hipLaunchKernelGGL((mttkrp_kind1<T, NT, true>), grid, block, 0, st, d);
    else hipLaunchKernelGGL((mttkrp_kind1<T, NT, false>), grid, block, 0, st, d);
  } else if (p.kind == 2) {
    if (vec) hipLaunchKernelGGL((mttkrp_kind23<T, NT, 2, false, true>), grid, block, 0, st, d);
    else hipLaunchKernelGGL((mttkrp_kind23<T, NT, 2, false, false>), grid, block, 0, st, d);
  } else {
    if (vec) hipLaunchKernelGGL((mttkrp_kind23<T, NT, 2, true, true>), grid, block, 0, st, d);
    else hipLaunchKernelGGL((mttkrp_kind23<T, NT, 2, true, false>), grid, block, 0, st, d);
  }
  return hipGetLastError();
}

hipError_t mttkrp_launch(const MttkrpPlan& p, const int64_t* dims, int N, int n, int R,
                         const void* z, bool fp32, const double* const* a64,
                         const float* const* a32, double* out, const PrepArgs* prep,
                         hipStream_t st) {
  MttkrpDesc d{};
  if (prep) {
    d.prep = 1;
    d.pa = *prep;
  }
  d.z = z;
  d.N = N;
  d.n = n;
  d.R = R;
  d.kind = p.kind;
  d.I0 = dims[0];
  d.I1 = dims[1];
  d.S = 1;
  for (int m = 2; m < N; ++m) d.S *= dims[m];
  d.In = dims[n];
  for (int m = 0; m < N; ++m) d.a64[m] = a64[m];
  const int kmode = (p.kind == 1) ? 1 : 0;
  d.ak = fp32 ? (const void*)a32[kmode] : (const void*)a64[kmode];
  d.out = out;
  d.ns = N - 2 > 0 ? N - 2 : 0;
  int64_t st_acc = 1;
  for (int j = 0; j < d.ns; ++j) {
    d.sext[j] = dims[j + 2];
    d.sst[j] = st_acc;
    st_acc *= dims[j + 2];
  }
  d.ngroups = p.ngroups;
  d.nsplit = p.nsplit;
  d.units = p.units;
  d.chunk = p.chunk;
  d.ksplit = p.ksplit;
  d.kchunk = p.kchunk;
  d.rgroups = p.rgroups;
  d.rest_count = (p.kind == 3) ? d.S / dims[n] : 0;
  // 4-wide vector loads need the contiguous extent to be a multiple of 4 and
  // an aligned base
  const size_t esz = fp32 ? 4 : 8;
  const bool vec = (dims[0] % 4 == 0) && (((uintptr_t)z) % (4 * esz) == 0);
  (void)esz;
  if (fp32) {
    return p.nt == 1 ? launch_typed<float, 1>(p, d, vec, st) : launch_typed<float, 2>(p, d, vec, st);
  }
  return p.nt == 1 ? launch_typed<double, 1>(p, d, vec, st) : launch_typed<double, 2>(p, d, vec, st);
}

}  // namespace cpamg

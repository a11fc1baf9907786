// Templates of the dense MTTKRP kernels, shared by the translation units that
// instantiate them (mttkrp.hip and the per-precision mttkrp_k_*.hip).
#pragma once
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

template <typename T, bool NTH>
__device__ __forceinline__ T ld(const T* p) {
  if (NTH) return __builtin_nontemporal_load(p);
  return *p;
}

// Load 4 consecutive entries p[0..3] (VEC: one 4-wide load).  Branch-free: an
// invalid entry (index >= nvalid) is loaded from `safe` (any valid, 16-byte
// aligned address); the consumer zeroes it with the validity mask, after the
// loads of the next step have been issued.
// NTH: non-temporal hint.  The tensor is streamed once per launch, but the
// hint only pays when one load instruction covers whole 128-byte lines; when a
// line is split over two instructions of a wave it is fetched twice.
template <typename T, bool VEC, bool NTH>
__device__ __forceinline__ typename Vec4<T>::type load4(const T* p, const T* __restrict__ safe,
                                                        int nvalid) {
  typedef typename Vec4<T>::type V;
  V v;
  if (VEC) {
    v = ld<V, NTH>(reinterpret_cast<const V*>(nvalid >= 4 ? p : safe));
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = ld<T, NTH>(nvalid > e ? p + e : safe);
  }
  return v;
}

// validity bits of one 4-wide load: bit e set when entry e is valid
template <bool VEC>
__device__ __forceinline__ uint32_t valid4(int nvalid) {
  if (VEC) return nvalid >= 4 ? 0xFu : 0u;
  return (1u << (nvalid < 0 ? 0 : (nvalid > 4 ? 4 : nvalid))) - 1u;
}

// VW consecutive entries (VW = 4 or 8) as one or two 4-wide loads; returns
// VW validity bits.
template <typename T, int VW, bool VEC, bool NTH>
__device__ __forceinline__ uint32_t loadw(const T* p, const T* __restrict__ safe, int nvalid,
                                          T (&out)[VW]) {
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < VW / 4; ++q) {
    const int nv = nvalid - 4 * q;
    const int nq = nv < 0 ? 0 : (nv > 4 ? 4 : nv);
    const typename Vec4<T>::type v = load4<T, VEC, NTH>(p + 4 * q, safe, nq);
    m |= valid4<VEC>(nq) << (4 * q);
#pragma unroll
    for (int e = 0; e < 4; ++e) out[4 * q + e] = v[e];
  }
  return m;
}

// The GEMM B operand (the contracted mode's factor, I x R) can be staged in
// LDS once per workgroup, transposed to Bs[c * ldb + i] for the 16*NT padded
// columns c; reads are then 4 consecutive i of one column per lane.  ldb pads
// the column stride so that the 16 columns read by one instruction fall into
// distinct banks; pad entries and columns c >= R hold zeros, and the last 4
// entries of every column are pad (a finite operand for masked lanes).
template <typename T> constexpr int64_t bstage_ld(int64_t I) {
  return (I + 3) / 4 * 4 + (sizeof(T) == 4 ? 4 : 6);
}
template <typename T> constexpr int64_t bstage_doubles(int64_t I, int NT) {
  return (16 * NT * bstage_ld<T>(I) * (int64_t)sizeof(T) + 7) / 8;
}

template <typename T, int NT>
__device__ __forceinline__ void stage_b(const T* __restrict__ ak, int I, int R, T* Bs) {
  constexpr int NC = 16 * NT;
  const int ldb = (int)bstage_ld<T>(I);
  const int tid = threadIdx.x;
  // zeros: the columns R..NC-1 (contiguous) and the pad rows i >= I of the others
  for (int e = tid; e < (NC - R) * ldb; e += kThreads) Bs[R * ldb + e] = T(0);
  const int pad = ldb - I;
  for (int e = tid; e < pad * R; e += kThreads) {
    const int c = e / pad;
    Bs[c * ldb + I + (e - c * pad)] = T(0);
  }
  // the factor is contiguous (I x R): coalesced loads, 16 in flight per thread
  // (one round trip up to 4096 entries); entry idx = i R + c goes to column c,
  // row i, with (i, c) stepped along with idx instead of divided out
  constexpr int SQ = 16;
  const int total = I * R;
  const int di = kThreads / R, dc = kThreads - di * R;
  for (int base = 0; base < total; base += SQ * kThreads) {
    T v[SQ];
#pragma unroll
    for (int j = 0; j < SQ; ++j) {
      const int idx = base + j * kThreads + tid;
      v[j] = ak[idx < total ? idx : 0];
    }
    int i = (base + tid) / R, c = base + tid - i * R;
#pragma unroll
    for (int j = 0; j < SQ; ++j) {
      if (base + j * kThreads + tid < total) Bs[c * ldb + i] = v[j];
      i += di;
      c += dc;
      if (c >= R) {
        c -= R;
        ++i;
      }
    }
  }
  __syncthreads();
}

typedef double d2 __attribute__((ext_vector_type(2)));
// 4 consecutive entries of Bs (16-byte aligned)
__device__ __forceinline__ void lds4(const float* p, float (&o)[4]) {
  const f4 v = *reinterpret_cast<const f4*>(p);
  o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
}
__device__ __forceinline__ void lds4(const double* p, double (&o)[4]) {
  const d2 v0 = *reinterpret_cast<const d2*>(p);
  const d2 v1 = *reinterpret_cast<const d2*>(p + 2);
  o[0] = v0[0]; o[1] = v0[1]; o[2] = v1[0]; o[3] = v1[1];
}

// One factor entry (GEMM B operand), 0 when !ok.
template <typename T>
__device__ __forceinline__ T loadb(const T* __restrict__ ak, int64_t idx, bool ok) {
  const T x = ak[ok ? idx : 0];
  return ok ? x : T(0);
}

// Product of the stripe-mode factors at stripe s, column col (skip mode `skip`).
// q = a / b, r = a % b for a >= 0, b >= 1 (wave-uniform): 32-bit division
// when a fits, which is far shorter than the 64-bit sequence
__device__ __forceinline__ void divmod(int64_t a, int64_t b, int64_t& q, int64_t& r) {
  if (b == 1) {
    q = a;
    r = 0;
  } else if (a <= 0x7fffffff && b <= 0x7fffffff) {
    const uint32_t qa = (uint32_t)a / (uint32_t)b;
    q = qa;
    r = a - (int64_t)qa * b;
  } else {
    q = a / b;
    r = a - q * b;
  }
}

// prod_{m >= 2, m != skip} A^(m)(s_m, col) for stripe s.  With one stripe mode
// (order 3) the entry is a plain load whose first use is at the end of the
// unit, so its latency hides under the tensor stream.
__device__ __forceinline__ double stripe_weight(const MttkrpDesc& d, int64_t s, int col, int skip) {
  if (d.ns == 1) return (col < d.R && skip != 2) ? d.a64[2][s * d.R + col] : (col < d.R ? 1.0 : 0.0);
  if (col >= d.R) return 0.0;
  double w = 1.0;
  for (int j = 0; j < d.ns; ++j) {
    const int m = j + 2;
    int64_t q, r, sj;
    divmod(s, d.sst[j], q, r);
    divmod(q, d.sext[j], r, sj);
    if (m != skip) w *= d.a64[m][sj * d.R + col];
  }
  return w;
}

// The same product as a loop over the stripe modes, each entry multiplied in
// as it arrives (the wait sits at the top of the unit).  Kinds 2 and 3 keep
// this form and the 64-bit index split except in one FP32 tile-storing
// variant: elsewhere the forms above cost registers (a wave per SIMD in
// several FP32 variants) or time (the FP64 mode-1 launch at 256^3 took 2 us
// longer).
__device__ __forceinline__ double stripe_weight_loop(const MttkrpDesc& d, int64_t s, int col, int skip) {
  if (col >= d.R) return 0.0;
  double w = 1.0;
  for (int j = 0; j < d.ns; ++j) {
    const int m = j + 2;
    const int64_t sj = (s / d.sst[j]) % d.sext[j];
    if (m != skip) w *= d.a64[m][sj * d.R + col];
  }
  return w;
}

// Workgroup 0 of a launch with prep set does the sweep bookkeeping for the
// update that follows (sweep.hpp), concurrently with the streaming workgroups;
// it is dispatched first, so it is resident from the start.
// NT: 16-column tiles of the kernel (R <= 16 NT); BATCH: batched launch
// (column groups).
template <int NT, bool BATCH>
__device__ __forceinline__ bool prep_block(const MttkrpDesc& d, int blk, double* smem) {
  if (!d.prep || blk != 0) return false;
  sweep_prep<8, 16 * NT, BATCH>(d.pa, smem, false);
  return true;
}

// LDS (doubles) of the streaming workgroups of each kernel
constexpr int kind1_smem() { return 4 * 16 * 2 * 16; }
constexpr int kind23_smem(int TW, int NT, bool k3) { return k3 ? 4 * 16 * NT : 4 * 16 * TW * 16 * NT; }

// ---------------------------------------------------------------------------
// kind 1: output mode 0.  Each lane loads VW consecutive rows i0 at one i1;
// sub-tile a holds rows i0 = grp*16*VW + VW*m + a (m = GEMM row).  Contraction
// over i1 on the matrix cores, Hadamard weight per stripe in FP64.
// ---------------------------------------------------------------------------
template <typename T, int NT, int VW, bool VEC, bool BL, bool BATCH = false>
__device__ __forceinline__ void kind1_body(const MttkrpDesc& d, int blk, double* smem) {
  typedef typename Vec4<T>::type V;
  constexpr int PANEL = 16 * VW;
  // 16 lanes x 16 bytes cover two whole lines only for 4-wide FP32 loads
  constexpr bool NTH = sizeof(T) == 4 && VW == 4;
  if (prep_block<NT, BATCH>(d, blk, smem)) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 15, g4 = lane >> 4;
  const int bid = blk - d.prep;
  const int grp = bid % d.ngroups;
  const int split = bid / d.ngroups;
  const T* __restrict__ z = reinterpret_cast<const T*>(d.z);
  const T* __restrict__ ak = reinterpret_cast<const T*>(d.ak);
  const int R = d.R;
  const int64_t I0 = d.I0, I1 = d.I1;
  const int64_t i0b = (int64_t)grp * PANEL + VW * r;   // first of this lane's VW rows
  const int64_t left = I0 - i0b;
  const int nrow = left <= 0 ? 0 : (left >= VW ? VW : (int)left);
  T* Bs = reinterpret_cast<T*>(smem);
  const int ldb = (int)bstage_ld<T>(I1);
  if (BL) stage_b<T, NT>(ak, (int)I1, R, Bs);

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
    int64_t s, kp;
    divmod(u, d.ksplit, s, kp);
    const int64_t kbeg = kp * d.kchunk;
    const int64_t kend = min(I1, kbeg + d.kchunk);
    double w[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) w[t] = stripe_weight(d, s, t * 16 + r, -1);
    V D[VW][NT];
#pragma unroll
    for (int a = 0; a < VW; ++a)
#pragma unroll
      for (int t = 0; t < NT; ++t) D[a][t] = V{0, 0, 0, 0};
    const T* zs = z + (size_t)s * I0 * I1 + i0b;
    // one step: 16 consecutive i1 (4 per lane group), VW rows per lane;
    // bit e*VW + a of the mask is set when zv[e][a] is a valid entry
    auto fetch = [&](int64_t k0, T (&zv)[4][VW], T (&b)[4][NT], uint32_t& mask) {
      mask = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i1 = k0 + 4 * g4 + e;
        const bool ok = i1 < kend;
        mask |= loadw<T, VW, VEC, NTH>(zs + i1 * I0, z, ok ? nrow : 0, zv[e]) << (e * VW);
        if (!BL) {
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const int col = t * 16 + r;
            b[e][t] = loadb(ak, i1 * R + col, ok && col < R);
          }
        }
      }
      if (BL) {
        // rows past kend read the zero pad at the end of the column
        const int64_t i1b = k0 + 4 * g4;
        const int boff = i1b < kend ? (int)i1b : ldb - 4;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          T b4[4];
          lds4(Bs + (t * 16 + r) * ldb + boff, b4);
#pragma unroll
          for (int e = 0; e < 4; ++e) b[e][t] = b4[e];
        }
      }
    };
    auto compute = [&](const T (&zv)[4][VW], const T (&b)[4][NT], uint32_t mask) {
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int a = 0; a < VW; ++a) {
          const T x = (mask >> (e * VW + a)) & 1u ? zv[e][a] : T(0);
#pragma unroll
          for (int t = 0; t < NT; ++t) D[a][t] = mma(x, b[e][t], D[a][t]);
        }
    };
    // two register buffers: the loads of the next step are in flight while
    // the matrix cores work on the current one (the scheduling barriers keep
    // each phase's loads ahead of the other buffer's matrix instructions)
    T zA[4][VW], zB[4][VW];
    T bA[4][NT], bB[4][NT];
    uint32_t mA, mB;
    fetch(kbeg, zA, bA, mA);
    int64_t k0 = kbeg;
    for (; k0 + 16 < kend; k0 += 32) {
      fetch(k0 + 16, zB, bB, mB);
      __builtin_amdgcn_sched_barrier(0);
      compute(zA, bA, mA);
      __builtin_amdgcn_sched_barrier(0);
      fetch(k0 + 32, zA, bA, mA);
      __builtin_amdgcn_sched_barrier(0);
      compute(zB, bB, mB);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (k0 < kend) compute(zA, bA, mA);
    // Hadamard-reduce with the stripe weight (FP64)
#pragma unroll
    for (int a = 0; a < VW; ++a)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[a][t][v] += (double)D[a][t][v] * w[t];
  }
  // deterministic cross-wave reduction through LDS, 2 sub-tiles x 16 columns
  // at a time: GEMM row m of sub-tile a holds i0 = grp*PANEL + VW*m + a
#pragma unroll
  for (int a0 = 0; a0 < VW; a0 += 2)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      __syncthreads();
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          smem[((wave * 16 + mfma_row<T>(g4, v)) * 2 + a) * 16 + r] = acc[a0 + a][t][v];
      __syncthreads();
      for (int idx = threadIdx.x; idx < 16 * 2 * 16; idx += kThreads) {
        const int q = idx / 16, c = idx % 16;   // q = 2*m + a
        const int m = q >> 1, a = q & 1;
        const int64_t i0 = (int64_t)grp * PANEL + VW * m + a0 + a;
        const int col = t * 16 + c;
        if (col < R && i0 < I0) {
          const double sum = smem[idx] + smem[512 + idx] + smem[1024 + idx] + smem[1536 + idx];
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
template <typename T, int NT, int TW, bool KIND3, int VW, bool VEC, bool BL, bool YS = false, bool BATCH = false>
__device__ __forceinline__ void kind23_body(const MttkrpDesc& d, int blk, double* smem) {
  typedef typename Vec4<T>::type V;
  constexpr int KC = 4 * VW;   // contraction chunk per step of the loop
  constexpr int ROWS = 16 * TW;
  if (prep_block<NT, BATCH>(d, blk, smem)) return;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = lane & 15, g4 = lane >> 4;
  const int bid = blk - d.prep;
  const int grp = bid % d.ngroups;
  const int split = bid / d.ngroups;
  const T* __restrict__ z = reinterpret_cast<const T*>(d.z);
  const T* __restrict__ ak = reinterpret_cast<const T*>(d.ak);
  const int R = d.R;
  const int64_t I0 = d.I0, I1 = d.I1;
  T* Bs = reinterpret_cast<T*>(smem);
  const int ldb = (int)bstage_ld<T>(I0);
  if (BL) stage_b<T, NT>(ak, (int)I0, R, Bs);

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
  // the early-issued stripe weight and the short index split only where they
  // cost no occupancy (the FP32 one-tile, two-row-tile, tile-storing kernel)
  constexpr bool EARLYW = sizeof(T) == 4 && YS && NT == 1 && TW == 2;
  const int64_t stride_n = KIND3 ? d.sst[jn] : 1;
  for (int64_t u = ubeg + wave; u < uend; u += 4) {
    int64_t uu, kp;
    if (EARLYW) {
      divmod(u, d.ksplit, uu, kp);
    } else {
      kp = u % d.ksplit;
      uu = u / d.ksplit;
    }
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
    for (int t = 0; t < NT; ++t)
      w[t] = EARLYW ? stripe_weight(d, s, t * 16 + r, KIND3 ? d.n : -1)
                    : stripe_weight_loop(d, s, t * 16 + r, KIND3 ? d.n : -1);
    // stage-2 operands are loaded before the contraction loop so that their
    // latency overlaps the tensor stream
    double a1w[KIND3 ? TW : 1][KIND3 ? NT : 1][4];
    if (KIND3) {
#pragma unroll
      for (int a = 0; a < TW; ++a)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t i1 = rowbase + a * 16 + mfma_row<T>(g4, v);
            const int col = t * 16 + r;
            a1w[a][t][v] = (i1 < I1 && col < R) ? d.a64[1][i1 * R + col] * w[t] : 0.0;
          }
    }
    V D[TW][NT];
#pragma unroll
    for (int a = 0; a < TW; ++a)
#pragma unroll
      for (int t = 0; t < NT; ++t) D[a][t] = V{0, 0, 0, 0};
    const T* zs = z + (size_t)s * I0 * I1;
    int64_t rowoff[TW];
    bool rowok[TW];
#pragma unroll
    for (int a = 0; a < TW; ++a) {
      const int64_t i1 = rowbase + a * 16 + r;
      rowok[a] = i1 < I1;
      rowoff[a] = (rowok[a] ? i1 : 0) * I0;
    }
    // one step: KC consecutive i0 (VW per lane group) for 16*TW rows i1;
    // bit a*VW + e of the mask is set when zv[a][e] is a valid entry
    auto fetch = [&](int64_t k0, T (&zv)[TW][VW], T (&b)[VW][NT], uint32_t& mask) {
      const int64_t kl = k0 + VW * g4;
      const int64_t nk = kend - kl;
      const int nval = nk >= VW ? VW : (nk > 0 ? (int)nk : 0);
      mask = 0;
#pragma unroll
      for (int a = 0; a < TW; ++a)
        mask |= loadw<T, VW, VEC, false>(zs + rowoff[a] + kl, z, rowok[a] ? nval : 0, zv[a]) << (a * VW);
      if (BL) {
        // entries past kend read the zero pad at the end of the column
        const int boff = nval ? (int)kl : ldb - 4;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int q = 0; q < VW / 4; ++q) {
            T b4[4];
            lds4(Bs + (t * 16 + r) * ldb + (nval > 4 * q ? boff + 4 * q : ldb - 4), b4);
#pragma unroll
            for (int e = 0; e < 4; ++e) b[4 * q + e][t] = b4[e];
          }
      } else {
#pragma unroll
        for (int e = 0; e < VW; ++e)
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const int col = t * 16 + r;
            b[e][t] = loadb(ak, (kl + e) * R + col, e < nval && col < R);
          }
      }
    };
    auto compute = [&](const T (&zv)[TW][VW], const T (&b)[VW][NT], uint32_t mask) {
#pragma unroll
      for (int e = 0; e < VW; ++e)
#pragma unroll
        for (int a = 0; a < TW; ++a) {
          const T x = (mask >> (a * VW + e)) & 1u ? zv[a][e] : T(0);
#pragma unroll
          for (int t = 0; t < NT; ++t) D[a][t] = mma(x, b[e][t], D[a][t]);
        }
    };
    T zA[TW][VW], zB[TW][VW];
    T bA[VW][NT], bB[VW][NT];
    uint32_t mA, mB;
    fetch(kbeg, zA, bA, mA);
    int64_t k0 = kbeg;
    for (; k0 + KC < kend; k0 += 2 * KC) {
      fetch(k0 + KC, zB, bB, mB);
      __builtin_amdgcn_sched_barrier(0);
      compute(zA, bA, mA);
      __builtin_amdgcn_sched_barrier(0);
      fetch(k0 + 2 * KC, zA, bA, mA);
      __builtin_amdgcn_sched_barrier(0);
      compute(zB, bB, mB);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (k0 < kend) compute(zA, bA, mA);
    // dimension tree: keep the stage-1 tile (complete: the contraction is not split)
    if (YS && !KIND3) {
#pragma unroll
      for (int a = 0; a < TW; ++a)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int64_t i1 = rowbase + a * 16 + mfma_row<T>(g4, v);
            const int col = t * 16 + r;
            if (i1 < I1 && col < R) {
              const size_t yi = ((size_t)s * I1 + i1) * R + col;
              if (sizeof(T) == 4) reinterpret_cast<float*>(d.y)[yi] = (float)D[a][t][v];
              else d.y[yi] = (double)D[a][t][v];
            }
          }
    }
    // Hadamard-reduce (FP64)
    if (KIND3) {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        double part = 0.0;
#pragma unroll
        for (int a = 0; a < TW; ++a)
#pragma unroll
          for (int v = 0; v < 4; ++v) part += (double)D[a][t][v] * a1w[a][t][v];
        acc[0][t][0] += part;
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
  __syncthreads();   // smem aliases the staged B operand
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

// (the FP32 one-tile, 4-wide variant with the factor in LDS is held at three waves per
// SIMD, which its streaming path fits without spills; left to itself the
// compiler takes a few more registers)
template <typename T, int NT, int VW, bool VEC, bool BL>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu((NT == 1 && VW == 4 && sizeof(T) == 4 && BL) ? 3 : 1)))
void mttkrp_kind1(MttkrpDesc d) {
  extern __shared__ double smem[];
  kind1_body<T, NT, VW, VEC, BL>(d, blockIdx.x, smem);
}

template <typename T, int NT, int TW, bool KIND3, int VW, bool VEC, bool BL, bool YS = false>
__global__ __launch_bounds__(kThreads) void mttkrp_kind23(MttkrpDesc d) {
  extern __shared__ double smem[];
  kind23_body<T, NT, TW, KIND3, VW, VEC, BL, YS>(d, blockIdx.x, smem);
}

// Kernel of a single-problem launch plan, per tensor precision and lane width
// (vec: 4-wide loads allowed; ys: mode-1 launch that also stores Y).
const void* mttkrp_kernel_f32v4(const MttkrpPlan& p, bool vec, bool ys);
const void* mttkrp_kernel_f32v8(const MttkrpPlan& p, bool vec, bool ys);
const void* mttkrp_kernel_f64(const MttkrpPlan& p, bool vec, bool ys);

}  // namespace cpamg

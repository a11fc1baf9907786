// Dense MTTKRP: batched and dimension-tree kernels, launch planning and dispatch.
// The kernel templates live in mttkrp_kernels.hpp; the per-precision
// instantiations of the single-problem kernels are compiled in mttkrp_k_*.hip.
#include "mttkrp_kernels.hpp"

namespace cpamg {

// Batched MTTKRPs (one mode of many problems in one launch): tile t runs
// workgroup tiles[t].y of the launch described by descs[tiles[t].x].  Every
// problem stages its contracted factor in LDS; 4-wide loads where the problem
// allows them.  Tiles of problems with nothing left in the current phase exit.
// (the FP32 mode-0 variant is held at the three waves per SIMD its streaming
// path fits, one register above which the bookkeeping path would push it)
template <typename T, int NT, int KIND>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu((NT == 1 && KIND == 1 && sizeof(T) == 4) ? 3 : 1)))
void mttkrp_batched(const MttkrpDesc* __restrict__ descs, const int2* __restrict__ tiles) {
  extern __shared__ double smem[];
  const int2 t = tiles[blockIdx.x];
  const MttkrpDesc& d = descs[t.x];
  if (d.pa.st && (!d.pa.st->active || d.pa.st->phase != d.pa.run_phase)) return;
  if (KIND == 1) {
    if (d.vec) kind1_body<T, NT, 4, true, true, true>(d, t.y, smem);
    else kind1_body<T, NT, 4, false, true, true>(d, t.y, smem);
  } else {
    if (d.vec) kind23_body<T, NT, 2, KIND == 3, 4, true, true, false, true>(d, t.y, smem);
    else kind23_body<T, NT, 2, KIND == 3, 4, false, true, false, true>(d, t.y, smem);
  }
}

// ---------------------------------------------------------------------------
// Dimension-tree MTTKRP of mode n >= 2 from Y (Y in the tensor's precision,
// everything else FP64).  Workgroup
// (row i_n, split) sums its chunk of rest indices q.  Lane layout: thread t
// owns column c = t % RM of the rows t / RM, t / RM + 256 / RM, ... of each
// Y block (Y[s] and A^(1) share the I1 x R row-major layout), so a wave reads
// 64 / RM whole rows per load.  The work is the flat sequence of (q, row step)
// pairs, KU of them per round with every load issued before the first use
// (indices clamped instead of branched).  Per chunk of up to kYQ rest indices
// the stripe offsets and the weights prod_{m >= 2, m != n} A^(m)(s_m, c) are
// staged in LDS first.  Column sums: across the lanes of a column in a fixed
// shuffle order, then the four waves in order.
// ---------------------------------------------------------------------------
constexpr int kYQ = 32;

template <int RM, bool Y32>
__global__ __launch_bounds__(kThreads) void ymttkrp_kernel(YDesc d) {
  extern __shared__ double smem[];
  if (d.prep && blockIdx.x == 0) {
    sweep_prep<16, RM>(d.pa, smem, false);
    return;
  }
  __shared__ double sw[kYQ * RM];        // weights of the chunk's rest indices
  __shared__ int64_t sbase[kYQ];         // Y offsets of their blocks
  __shared__ double swave[4 * RM];       // per-wave column sums
  constexpr int RPW = kThreads / RM;     // rows per round of the workgroup
  constexpr int KU = 16;                 // (q, row step) pairs per round
  const int bid = blockIdx.x - d.prep;
  const int64_t row = bid % d.In;
  const int split = (int)(bid / d.In);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R = d.R;
  const int I1 = (int)d.I1;
  const int jn = d.n - 2;
  const int c = tid % RM, rl = tid / RM;
  const bool cok = c < R;
  const int cc = cok ? c : 0;
  const int64_t qbeg = (int64_t)split * d.rchunk;
  const int64_t qend = min(d.rest_count, qbeg + d.rchunk);
  const int steps = (I1 + RPW - 1) / RPW;   // row steps per rest index
  const double* __restrict__ a1 = d.a64[1];
  const double* __restrict__ y = d.y;
  const float* __restrict__ y32 = reinterpret_cast<const float*>(d.y);
  double acc = 0.0;
  for (int64_t q0 = qbeg; q0 < qend; q0 += kYQ) {
    const int nq = (int)min<int64_t>(kYQ, qend - q0);
    // stripe offsets and weights of rest indices q0 .. q0 + nq - 1
    __syncthreads();
    for (int e = tid; e < nq * RM; e += kThreads) {
      const int qi = e / RM, col = e % RM;
      int64_t s = row * d.sst[jn], qq = q0 + qi;
      double w = col < R ? 1.0 : 0.0;
      for (int j = 0; j < d.ns; ++j) {
        if (j == jn) continue;
        const int64_t sj = qq % d.sext[j];
        qq /= d.sext[j];
        s += sj * d.sst[j];
        if (col < R) w *= d.a64[j + 2][sj * R + col];
      }
      sw[qi * RM + col] = w;
      if (col == 0) sbase[qi] = s * d.I1 * R;
    }
    __syncthreads();
    const int T = nq * steps;
    int qi = 0, st = 0;   // (q, step) of the round's first pair
    for (int t0 = 0; t0 < T; t0 += KU) {
      double yv[KU], av[KU], wv[KU];
      int qk = qi, sk = st;
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int i1 = sk * RPW + rl;
        const bool v = (t0 + u < T) && cok && i1 < I1;
        const int qs = qk < nq ? qk : nq - 1;
        const int64_t ar = (int64_t)(v ? i1 : 0) * R + cc;
        yv[u] = Y32 ? (double)y32[sbase[qs] + ar] : y[sbase[qs] + ar];
        av[u] = a1[ar];
        wv[u] = v ? sw[qs * RM + c] : 0.0;
        if (++sk == steps) {
          sk = 0;
          ++qk;
        }
      }
#pragma unroll
      for (int u = 0; u < KU; ++u) acc = fma(wv[u] * yv[u], av[u], acc);
      qi = qk;
      st = sk;
    }
  }
  // column sums: lanes c, c + RM, ... of the wave (fixed order), then the waves
#pragma unroll
  for (int off = RM; off < 64; off <<= 1) acc += __shfl_xor(acc, off);
  if (lane < RM) swave[wave * RM + lane] = acc;
  __syncthreads();
  if (tid < R) {
    const double x = ((swave[tid] + swave[RM + tid]) + swave[2 * RM + tid]) + swave[3 * RM + tid];
    d.out[((size_t)split * d.In + row) * R + tid] = x;
  }
}

int ymttkrp_nsplit(const int64_t* dims, int N, int n, int R) {
  (void)R;
  int64_t S = 1;
  for (int m = 2; m < N; ++m) S *= dims[m];
  const int64_t rest = S / dims[n];
  // aim for about two workgroups per compute unit over all output rows
  const int64_t want = std::max<int64_t>(1, 512 / std::max<int64_t>(1, dims[n]));
  return (int)std::max<int64_t>(1, std::min<int64_t>(rest, want));
}

hipError_t ymttkrp_launch(const int64_t* dims, int N, int n, int R, const double* y, bool y32,
                          const double* const* a64, double* out, int nsplit, const PrepArgs* prep,
                          hipStream_t st) {
  YDesc d{};
  d.y = y;
  d.y32 = y32 ? 1 : 0;
  for (int m = 0; m < N; ++m) d.a64[m] = a64[m];
  d.out = out;
  d.I1 = dims[1];
  d.S = 1;
  for (int m = 2; m < N; ++m) d.S *= dims[m];
  d.In = dims[n];
  d.N = N;
  d.n = n;
  d.R = R;
  d.ns = N - 2;
  int64_t acc = 1;
  for (int j = 0; j < d.ns; ++j) {
    d.sext[j] = dims[j + 2];
    d.sst[j] = acc;
    acc *= dims[j + 2];
  }
  d.rest_count = d.S / d.In;
  d.nsplit = nsplit;
  d.rchunk = (d.rest_count + nsplit - 1) / nsplit;
  d.prep = prep ? 1 : 0;
  if (prep) {
    d.pa = *prep;
    d.pa.lds = prep_smem_doubles(N, R);
  }
  const size_t smem = prep ? sizeof(double) * (size_t)prep_smem_doubles(N, R) : 0;
  dim3 grid((unsigned)(d.In * nsplit + d.prep)), block(kThreads);
  if (R <= 16) {
    if (y32) hipLaunchKernelGGL((ymttkrp_kernel<16, true>), grid, block, smem, st, d);
    else hipLaunchKernelGGL((ymttkrp_kernel<16, false>), grid, block, smem, st, d);
  } else {
    if (y32) hipLaunchKernelGGL((ymttkrp_kernel<32, true>), grid, block, smem, st, d);
    else hipLaunchKernelGGL((ymttkrp_kernel<32, false>), grid, block, smem, st, d);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// host side: planning and dispatch
// ---------------------------------------------------------------------------
static int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

MttkrpPlan mttkrp_plan(int N, const int64_t* dims, int n, int R, bool fp32, const PlanOpts& o) {
  MttkrpPlan p{};
  const int64_t I0 = dims[0], I1 = dims[1];
  int64_t S = 1;
  for (int m = 2; m < N; ++m) S *= dims[m];
  // consecutive tensor entries per lane load: 4 (FP64: 32 bytes), 4 or 8 (FP32)
  const int64_t vw = (fp32 && o.vw == 8) ? 8 : 4;
  p.vw = (int32_t)vw;
  p.nt = R <= 16 ? 1 : 2;
  p.tw = (o.tw == 4 && p.nt == 1) ? 4 : 2;
  const int64_t rows = 16 * p.tw;
  const int64_t target = std::max<int64_t>(1, o.target_wgs);
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
  // split the contraction when there are too few (group, unit) pairs: aim for
  // four units (one per wave) in each of `target` workgroups
  const int64_t kchunks = ceil_div(K, kgran);
  int64_t ks = o.ksplit;
  if (ks <= 0) {
    ks = 1;
    if ((int64_t)p.ngroups * base_units < target * 4)
      ks = ceil_div(target * 4, (int64_t)p.ngroups * base_units);
  }
  ks = std::max<int64_t>(1, std::min<int64_t>(ks, kchunks));
  int64_t kchunk = ceil_div(kchunks, ks) * kgran;
  // FP32 accumulates one contraction piece in the matrix cores and adds the
  // pieces in FP64: pieces of at most 256 keep the error within 256 u32
  while (fp32 && kchunk > 256 && ks < kchunks) kchunk = ceil_div(kchunks, ++ks) * kgran;
  ks = ceil_div(K, kchunk);
  p.ksplit = (int32_t)ks;
  p.kchunk = (int32_t)kchunk;
  p.units = base_units * ks;
  // units per workgroup: a multiple of 4 so the four waves stay balanced
  const int64_t nsplit_max = std::max<int64_t>(1, target / p.ngroups);
  int64_t chunk = ceil_div(p.units, nsplit_max);
  // a multiple of 4 units keeps the four waves of a workgroup balanced; it is
  // used when it keeps at least 3/4 of the workgroups
  if (p.units >= 4) {
    const int64_t c4 = ceil_div(chunk, 4) * 4;
    if (4 * ceil_div(p.units, c4) >= 3 * ceil_div(p.units, chunk)) chunk = c4;
  }
  p.chunk = chunk;
  p.nsplit = (int32_t)ceil_div(p.units, p.chunk);
  p.partial_doubles = (size_t)p.nsplit * dims[n] * R;
  // stage the contracted factor (I1 x R for kind 1, I0 x R otherwise) in LDS
  // when it takes at most 64 KB
  const int64_t Ik = p.kind == 1 ? I1 : I0;
  p.bstage_doubles = fp32 ? bstage_doubles<float>(Ik, p.nt) : bstage_doubles<double>(Ik, p.nt);
  p.bl = (!o.nostage && p.bstage_doubles * 8 <= 64 * 1024) ? 1 : 0;
  if (!p.bl) p.bstage_doubles = 0;
  p.opts = o;
  return p;
}

static const void* select_kernel(const MttkrpPlan& p, bool fp32, bool vec, bool ys = false) {
  if (fp32) return p.vw == 8 ? mttkrp_kernel_f32v8(p, vec, ys) : mttkrp_kernel_f32v4(p, vec, ys);
  return mttkrp_kernel_f64(p, vec, ys);
}

// dynamic LDS bytes of a launch
size_t mttkrp_smem_bytes(const MttkrpPlan& p, int N, int R, bool prep) {
  int64_t d = p.kind == 1 ? kind1_smem() : kind23_smem(p.tw, p.nt, p.kind == 3);
  if (p.bl) d = std::max<int64_t>(d, p.bstage_doubles);
  // the bookkeeping workgroup works within the streaming workgroups' LDS; it
  // stages the stored Grams too when that needs at most 16 KB or no more
  // than the streaming workgroups use anyway
  if (prep) {
    const int64_t full = prep_smem_doubles(N, R);
    d = std::max<int64_t>(d, full <= std::max<int64_t>(d, 2048) ? full : prep_min_doubles(N, R));
  }
  return sizeof(double) * (size_t)d;
}

int mttkrp_capacity(const MttkrpPlan& p, bool fp32) {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
  }
  const void* k = select_kernel(p, fp32, true);
  int nb = 0;
  const size_t smem = mttkrp_smem_bytes(p, 8, kMaxRank, false);
  if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kThreads, smem) != hipSuccess || nb < 1)
    nb = 1;
  return nb * cus;
}

template <typename T, int NT>
static const void* batched_ptr(int kind) {
  if (kind == 1) return (const void*)mttkrp_batched<T, NT, 1>;
  if (kind == 2) return (const void*)mttkrp_batched<T, NT, 2>;
  return (const void*)mttkrp_batched<T, NT, 3>;
}

hipError_t mttkrp_batched_launch(int kind, bool fp32, int nt, const MttkrpDesc* descs,
                                 const int2* tiles, int ntiles, size_t smem_bytes, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  const void* k = fp32 ? (nt == 1 ? batched_ptr<float, 1>(kind) : batched_ptr<float, 2>(kind))
                       : (nt == 1 ? batched_ptr<double, 1>(kind) : batched_ptr<double, 2>(kind));
  void* args[] = {(void*)&descs, (void*)&tiles};
  return hipLaunchKernel(k, dim3((unsigned)ntiles), dim3(kThreads), args, smem_bytes, st);
}

hipError_t mttkrp_launch(const MttkrpPlan& p, const int64_t* dims, int N, int n, int R,
                         const void* z, bool fp32, const double* const* a64,
                         const float* const* a32, double* out, const PrepArgs* prep,
                         hipStream_t st, double* y) {
  if (y && (p.kind != 2 || p.ksplit != 1)) return hipErrorInvalidValue;
  MttkrpDesc d = mttkrp_desc(p, dims, N, n, R, z, fp32, a64, a32, out, prep, y);
  const void* k = select_kernel(p, fp32, d.vec != 0, y != nullptr);
  if (!k) return hipErrorInvalidValue;
  dim3 grid((unsigned)((int64_t)p.ngroups * p.nsplit + (d.prep ? 1 : 0))), block(kThreads);
  void* args[] = {&d};
  return hipLaunchKernel(k, grid, block, args, mttkrp_smem_bytes(p, N, R, d.prep != 0), st);
}

MttkrpDesc mttkrp_desc(const MttkrpPlan& p, const int64_t* dims, int N, int n, int R,
                       const void* z, bool fp32, const double* const* a64,
                       const float* const* a32, double* out, const PrepArgs* prep, double* y) {
  MttkrpDesc d{};
  d.y = y;
  if (prep) {
    d.prep = 1;
    d.pa = *prep;
    d.pa.lds = (int32_t)(mttkrp_smem_bytes(p, N, R, true) / sizeof(double));
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
  d.vec = ((dims[0] % 4 == 0) && (((uintptr_t)z) % (4 * esz) == 0)) ? 1 : 0;
  return d;
}

}  // namespace cpamg

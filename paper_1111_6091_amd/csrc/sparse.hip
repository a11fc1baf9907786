// Sparse finest level (Section 6.2): MTTKRP over the stored entries, the
// scatter that turns a sparse tensor into a dense one for the restriction,
// and the host-side per-mode orderings.
//
// The MTTKRP of mode n reads each stored entry once (its indices, its value)
// and gathers one factor row per other mode: about N R nnz multiply-adds, the
// cost the paper gives for a sparse relaxation.  Output rows are owned by
// workgroups (the entries of one mode-n index are contiguous in perm[n]), so
// the sums need no atomics and repeat bit for bit; a long row is split over
// several workgroups whose partial sums the epilogue adds in a fixed order.
#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"
#include "sweep.hpp"

namespace cpamg {

namespace {

struct SpMttkrpDesc {
  SpTensor t;
  const double* a64[kMaxOrder];
  double* out;      // [nsplit][I_n][R]
  int64_t In;
  int32_t n, R, nsplit;
  int32_t prep;
  PrepArgs pa;
};

template <int RM>
__global__ __launch_bounds__(kThreads) void sp_mttkrp_kernel(SpMttkrpDesc d) {
  extern __shared__ double smem[];
  if (d.prep && blockIdx.x == 0) {
    sweep_prep<16, RM>(d.pa, smem, false);
    return;
  }
  const int bid = blockIdx.x - d.prep;
  const int64_t row = bid % d.In;
  const int split = (int)(bid / d.In);
  const int tid = threadIdx.x;
  const int N = d.t.N, n = d.n, R = d.R;
  const int64_t beg = d.t.rowptr[n][row], end = d.t.rowptr[n][row + 1];
  const int64_t ch = (end - beg + d.nsplit - 1) / d.nsplit;
  const int64_t kb = beg + (int64_t)split * ch;
  const int64_t ke = min(end, kb + ch);
  const int32_t* __restrict__ perm = d.t.perm[n];
  const int32_t* __restrict__ idx = d.t.idx;
  const double* __restrict__ vals = d.t.vals;
  double acc[RM];
#pragma unroll
  for (int r = 0; r < RM; ++r) acc[r] = 0.0;
  for (int64_t k = kb + tid; k < ke; k += kThreads) {
    const int64_t id = perm[k];
    const int32_t* ix = idx + id * N;
    const double v = vals[id];
    double w[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) w[r] = v;
    for (int m = 0; m < N; ++m) {
      if (m == n) continue;
      const double* am = d.a64[m] + (int64_t)ix[m] * R;
#pragma unroll
      for (int r = 0; r < RM; ++r)
        if (r < R) w[r] *= am[r];
    }
#pragma unroll
    for (int r = 0; r < RM; ++r) acc[r] += w[r];
  }
  // block reduction through LDS, 16 columns at a time, in a fixed order:
  // 16 consecutive threads' values, then the 16 part sums
#pragma unroll
  for (int c0 = 0; c0 < RM; c0 += 16) {
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) smem[c * kThreads + tid] = acc[c0 + c];
    __syncthreads();
    {
      const int c = tid >> 4, part = tid & 15;
      double x = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) x += smem[c * kThreads + part * 16 + i];
      smem[16 * kThreads + tid] = x;
    }
    __syncthreads();
    if (tid < 16 && c0 + tid < R) {
      double x = 0.0;
#pragma unroll
      for (int i = 0; i < 16; ++i) x += smem[16 * kThreads + tid * 16 + i];
      d.out[((int64_t)split * d.In + row) * R + c0 + tid] = x;
    }
  }
}

__global__ __launch_bounds__(kThreads) void sp_densify_kernel(SpTensor t, double* dense) {
  int64_t st[kMaxOrder];
  int64_t acc = 1;
  for (int m = 0; m < t.N; ++m) {
    st[m] = acc;
    acc *= t.dims[m];
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < t.nnz; k += stride) {
    const int32_t* ix = t.idx + k * t.N;
    int64_t lin = 0;
    for (int m = 0; m < t.N; ++m) lin += (int64_t)ix[m] * st[m];
    dense[lin] = t.vals[k];
  }
}

}  // namespace

int sp_mttkrp_nsplit(const SpTensor& t, int n) {
  const int64_t In = t.dims[n];
  const int64_t avg = (t.nnz + In - 1) / In;
  // about 1024 workgroups over all rows, but at least one entry per thread
  const int64_t want = std::max<int64_t>(1, 1024 / In);
  const int64_t cap = std::max<int64_t>(1, avg / kThreads);
  return (int)std::max<int64_t>(1, std::min(want, cap));
}

hipError_t sp_mttkrp_launch(const SpTensor& t, int n, int R, const double* const* a64, double* out,
                            int nsplit, const PrepArgs* prep, hipStream_t st) {
  SpMttkrpDesc d{};
  d.t = t;
  for (int m = 0; m < t.N; ++m) d.a64[m] = a64[m];
  d.out = out;
  d.In = t.dims[n];
  d.n = n;
  d.R = R;
  d.nsplit = nsplit;
  d.prep = prep ? 1 : 0;
  if (prep) {
    d.pa = *prep;
    d.pa.lds = prep_smem_doubles(t.N, R);
  }
  const size_t smem =
      sizeof(double) * (size_t)std::max(17 * kThreads, prep ? prep_smem_doubles(t.N, R) : 0);
  dim3 grid((unsigned)(d.In * nsplit + d.prep)), block(kThreads);
  if (R <= 16) hipLaunchKernelGGL(sp_mttkrp_kernel<16>, grid, block, smem, st, d);
  else hipLaunchKernelGGL(sp_mttkrp_kernel<32>, grid, block, smem, st, d);
  return hipGetLastError();
}

hipError_t sp_densify_launch(const SpTensor& t, double* dense, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>((t.nnz + kThreads - 1) / kThreads, 8192);
  hipLaunchKernelGGL(sp_densify_kernel, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(kThreads), 0, st,
                     t, dense);
  return hipGetLastError();
}

cp_status sparse_index_host(int order, const int64_t* dims, int64_t nnz, const int32_t* idx,
                            int64_t* rowptr, int32_t* perm, std::string* msg) {
  if (order < 2 || order > kMaxOrder) {
    *msg = "order outside [2, " + std::to_string(kMaxOrder) + "]";
    return CP_ERR_SHAPE;
  }
  if (nnz < 1 || nnz > INT32_MAX) {
    *msg = "nnz " + std::to_string(nnz) + " outside [1, 2^31 - 1]";
    return CP_ERR_SHAPE;
  }
  for (int m = 0; m < order; ++m)
    if (dims[m] < 1 || dims[m] > (int64_t(1) << 31)) {
      *msg = "dims[" + std::to_string(m) + "] out of range";
      return CP_ERR_SHAPE;
    }
  for (int64_t k = 0; k < nnz; ++k)
    for (int m = 0; m < order; ++m) {
      const int32_t i = idx[k * order + m];
      if (i < 0 || i >= dims[m]) {
        *msg = "entry " + std::to_string(k) + ": index " + std::to_string(i) + " outside mode " +
               std::to_string(m) + "'s extent";
        return CP_ERR_INVALID;
      }
    }
  // no index tuple twice: sort the ids by tuple, compare neighbours
  std::vector<int32_t> ord(nnz);
  std::iota(ord.begin(), ord.end(), 0);
  auto tuple_less = [&](int32_t a, int32_t b) {
    for (int m = order - 1; m >= 0; --m) {
      const int32_t x = idx[(int64_t)a * order + m], y = idx[(int64_t)b * order + m];
      if (x != y) return x < y;
    }
    return false;
  };
  std::sort(ord.begin(), ord.end(), tuple_less);
  for (int64_t k = 1; k < nnz; ++k)
    if (!tuple_less(ord[k - 1], ord[k])) {
      *msg = "entries " + std::to_string(ord[k - 1]) + " and " + std::to_string(ord[k]) +
             " store the same index tuple";
      return CP_ERR_INVALID;
    }
  // counting sort per mode (stable: ids increase within an index)
  int64_t* rp = rowptr;
  for (int m = 0; m < order; ++m) {
    const int64_t I = dims[m];
    std::vector<int64_t> cnt(I + 1, 0);
    for (int64_t k = 0; k < nnz; ++k) ++cnt[idx[k * order + m] + 1];
    for (int64_t i = 0; i < I; ++i) cnt[i + 1] += cnt[i];
    std::copy(cnt.begin(), cnt.end(), rp);
    int32_t* pm = perm + (int64_t)m * nnz;
    for (int64_t k = 0; k < nnz; ++k) pm[cnt[idx[k * order + m]]++] = (int32_t)k;
    rp += I + 1;
  }
  return CP_OK;
}

}  // namespace cpamg

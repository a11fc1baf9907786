// C ABI of libcpamg: argument checking, workspace and launch sequencing.
// Every compute call validates its arguments on the host, sizes the workspace,
// then only enqueues kernels on the context's stream.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <limits>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace cpamg;

namespace {

constexpr int kTargetWgs = 512;
constexpr int kNumCounters = 16;
enum CounterId { CNT_EPI = 0, CNT_RES = 1, CNT_DOT = 2, CNT_DOT2 = 3 };

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// Scratch of the allocation-free entry point (cp_mttkrp_noalloc): the per-split
// MTTKRP partial sums.  Each device holds its own copy of the array for the
// life of the process.  In host code the array's name is not a device address:
// host code uses only the address that hipGetSymbolAddress returned for the
// device (g_scratch[device]), looked up once per device in cp_ctx_create.
static __device__ __align__(256) double scratch[CP_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Address of this device's scratch array (the device is current); looked up on
// the first call per device.
hipError_t scratch_lookup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch[device] = ptr;
  return hipSuccess;
}

}  // namespace

struct cp_ctx_s {
  hipStream_t stream = nullptr;
  int device = 0;
  std::string err;
  char* ws = nullptr;
  size_t ws_cap = 0;
  // fixed region: counters, flags, factorization of Gamma, scalars
  char* fixed = nullptr;
  int32_t* counters = nullptr;
  uint32_t* flags = nullptr;
  double* prep_out = nullptr;   // Gamma factor + column scales for the next update
  int32_t* chol_kind = nullptr;
  double* scal = nullptr;   // 64 scratch scalars
  // sweeps of order >= 3 reuse the mode-1 stage-1 tiles for modes >= 2
  int dimtree = 1;
  // CP-FAS V-cycles are recorded once into a HIP graph per argument set and
  // replayed (CP_OPT_GRAPHS); capture runs on a private stream
  int graphs = 1;
  // relaxations of small levels in one workgroup (CP_OPT_SMALL_LEVELS)
  int small = 1;
  hipStream_t cap_stream = nullptr;
  std::map<std::string, hipGraphExec_t> gcache;
  // launch configurations of the MTTKRP kernels: tuned options and plan cache
  std::map<std::string, PlanOpts> tuned;
  std::map<std::string, MttkrpPlan> plans;
  std::string plans_text;
  // optional per-launch event timing
  bool prof = false;
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
};

namespace {

cp_status set_err(cp_ctx c, cp_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

cp_status hip_check(cp_ctx c, hipError_t e, const char* what) {
  if (e != hipSuccess) return set_err(c, CP_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return CP_OK;
}

#define HIPCHK(expr)                                        \
  do {                                                      \
    cp_status _s = hip_check(ctx, (expr), #expr);           \
    if (_s != CP_OK) return _s;                             \
  } while (0)

// Event pair around one launch when profiling is on.
struct ProfScope {
  cp_ctx ctx;
  int cls;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(cp_ctx c, int k) : ctx(c), cls(k) {
    if (!ctx->prof) return;
    a = take();
    b = take();
    if (a) (void)hipEventRecord(a, ctx->stream);
  }
  hipEvent_t take() {
    if (!ctx->pool.empty()) {
      hipEvent_t e = ctx->pool.back();
      ctx->pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~ProfScope() {
    if (!ctx->prof || !a || !b) return;
    (void)hipEventRecord(b, ctx->stream);
    ctx->recs.push_back({cls, a, b});
  }
};

// Grow the workspace to at least `bytes` (synchronizes the stream first).
// Drop the recorded graphs (they hold workspace addresses).
void clear_graphs(cp_ctx ctx) {
  for (auto& kv : ctx->gcache) (void)hipGraphExecDestroy(kv.second);
  ctx->gcache.clear();
}

cp_status ensure_ws(cp_ctx ctx, size_t bytes) {
  if (bytes <= ctx->ws_cap) return CP_OK;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  clear_graphs(ctx);
  if (ctx->ws) HIPCHK(hipFree(ctx->ws));
  ctx->ws = nullptr;
  ctx->ws_cap = 0;
  size_t cap = std::max(bytes, size_t(1) << 20);
  hipError_t e = hipMalloc((void**)&ctx->ws, cap);
  if (e != hipSuccess) return set_err(ctx, CP_ERR_NOMEM, "workspace of %zu bytes: %s", cap, hipGetErrorString(e));
  ctx->ws_cap = cap;
  return CP_OK;
}

struct Arena {
  char* base;
  size_t off = 0;
  explicit Arena(char* b) : base(b) {}
  template <typename T> T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off += align_up(count * sizeof(T));
    return p;
  }
};

// sizes-only pass of the same carving
struct Sizer {
  size_t off = 0;
  template <typename T> T* take(size_t count) {
    off += align_up(count * sizeof(T));
    return nullptr;
  }
};

int64_t numel(const cp_tensor* Z) {
  int64_t p = 1;
  for (int m = 0; m < Z->order; ++m) p *= Z->dims[m];
  return p;
}

bool is_sparse(const cp_tensor* Z) { return Z->nnz > 0; }

SpTensor sp_view(const cp_tensor* Z) {
  SpTensor t{};
  t.N = Z->order;
  t.nnz = Z->nnz;
  t.idx = Z->idx;
  t.vals = Z->vals;
  for (int m = 0; m < Z->order; ++m) {
    t.dims[m] = Z->dims[m];
    t.rowptr[m] = Z->rowptr[m];
    t.perm[m] = Z->perm[m];
  }
  return t;
}

cp_status check_ctx(cp_ctx ctx) { return ctx ? CP_OK : CP_ERR_INVALID; }

cp_status check_tensor(cp_ctx ctx, const cp_tensor* Z, bool need64, bool need32, const char* name) {
  if (!Z) return set_err(ctx, CP_ERR_INVALID, "%s is NULL", name);
  if (Z->order < 2 || Z->order > CP_MAX_ORDER)
    return set_err(ctx, CP_ERR_SHAPE, "%s: order %d outside [2, %d]", name, Z->order, CP_MAX_ORDER);
  for (int m = 0; m < Z->order; ++m)
    if (Z->dims[m] < 1 || Z->dims[m] > (int64_t(1) << 31))
      return set_err(ctx, CP_ERR_SHAPE, "%s: dims[%d] = %lld out of range", name, m, (long long)Z->dims[m]);
  if (Z->nnz < 0) return set_err(ctx, CP_ERR_SHAPE, "%s: nnz < 0", name);
  if (Z->nnz > 0) {
    if (need32)
      return set_err(ctx, CP_ERR_UNSUPPORTED, "%s: the sparse form is FP64 only (no CP_MIXED)", name);
    if (Z->nnz > INT32_MAX) return set_err(ctx, CP_ERR_SHAPE, "%s: nnz above 2^31 - 1", name);
    if (!Z->idx || !Z->vals) return set_err(ctx, CP_ERR_INVALID, "%s: sparse idx or vals is NULL", name);
    for (int m = 0; m < Z->order; ++m)
      if (!Z->rowptr[m] || !Z->perm[m])
        return set_err(ctx, CP_ERR_INVALID, "%s: sparse rowptr[%d] or perm[%d] is NULL", name, m, m);
    return CP_OK;
  }
  if (need64 && !Z->z64) return set_err(ctx, CP_ERR_INVALID, "%s: z64 is NULL", name);
  if (need32 && !Z->z32) return set_err(ctx, CP_ERR_INVALID, "%s: z32 is NULL (CP_MIXED needs the FP32 shadow)", name);
  return CP_OK;
}

cp_status require_dense(cp_ctx ctx, const cp_tensor* Z, const char* what) {
  if (Z && Z->nnz > 0) return set_err(ctx, CP_ERR_UNSUPPORTED, "%s: the sparse form is not supported here", what);
  return CP_OK;
}

cp_status check_factors(cp_ctx ctx, const cp_factors* A, int N, bool need32, const char* name) {
  if (!A) return set_err(ctx, CP_ERR_INVALID, "%s is NULL", name);
  if (A->rank < 1 || A->rank > CP_MAX_RANK)
    return set_err(ctx, CP_ERR_SHAPE, "%s: rank %d outside [1, %d]", name, A->rank, CP_MAX_RANK);
  for (int m = 0; m < N; ++m) {
    if (!A->a[m]) return set_err(ctx, CP_ERR_INVALID, "%s: a[%d] is NULL", name, m);
    if (need32 && !A->a32[m])
      return set_err(ctx, CP_ERR_INVALID, "%s: a32[%d] is NULL (CP_MIXED needs FP32 shadows)", name, m);
  }
  return CP_OK;
}

cp_status check_prec(cp_ctx ctx, cp_prec p) {
  if (p != CP_FP64 && p != CP_MIXED) return set_err(ctx, CP_ERR_INVALID, "unknown precision %d", (int)p);
  return CP_OK;
}

// Enqueue M^(n) partials for tensor Z (precision prec); returns the plan.
cp_status enqueue_mttkrp(cp_ctx ctx, const int64_t* dims, int N, int n, int R, const void* z,
                         bool fp32, const double* const* a64, const float* const* a32,
                         const MttkrpPlan& plan, double* out, const PrepArgs* prep = nullptr,
                         const SpTensor* sp = nullptr) {
  if (plan.kind == kSparseKind) {
    if (!sp) return set_err(ctx, CP_ERR_INVALID, "internal: sparse plan without a sparse tensor");
    ProfScope ps(ctx, CP_PROF_MTTKRP_MODE0_F64 + std::min(n, 2));
    HIPCHK(sp_mttkrp_launch(*sp, n, R, a64, out, plan.nsplit, prep, ctx->stream));
    return CP_OK;
  }
  ProfScope ps(ctx, (fp32 ? CP_PROF_MTTKRP_MODE0_F32 : CP_PROF_MTTKRP_MODE0_F64) + (plan.kind - 1));
  HIPCHK(mttkrp_launch(plan, dims, N, n, R, z, fp32, a64, a32, out, prep, ctx->stream));
  return CP_OK;
}

cp_status enqueue_epi(cp_ctx ctx, const EpiDesc& d) {
  ProfScope ps(ctx, d.op == EPI_UPDATE ? CP_PROF_UPDATE : CP_PROF_EPILOGUE_OTHER);
  HIPCHK(epi_launch(d, ctx->stream));
  return CP_OK;
}

cp_status enqueue_gram(cp_ctx ctx, double* const* A, float* const* A32, const int64_t* dims, int N,
                       int R, double* grams, double* sigma = nullptr) {
  ProfScope ps(ctx, CP_PROF_GRAM);
  HIPCHK(gram_launch(A, A32, dims, N, R, grams, ctx->stream, sigma));
  return CP_OK;
}

#define TRY(expr)                   \
  do {                              \
    cp_status _t = (expr);          \
    if (_t != CP_OK) return _t;     \
  } while (0)

std::string plan_key(int N, const int64_t* dims, int n, int R, bool fp32) {
  std::ostringstream o;
  o << "N=" << N << ";dims=";
  for (int m = 0; m < N; ++m) o << (m ? "," : "") << dims[m];
  o << ";n=" << n << ";R=" << R << ";prec=" << (fp32 ? "mixed" : "fp64");
  return o.str();
}

// Launch configuration for the MTTKRP of mode n: the tuned options when the
// autotuner (or an imported plan set) has seen this shape, otherwise as many
// streaming workgroups as stay resident next to the bookkeeping workgroup.
MttkrpPlan find_plan(cp_ctx ctx, int N, const int64_t* dims, int n, int R, bool fp32) {
  const std::string key = plan_key(N, dims, n, R, fp32);
  auto hit = ctx->plans.find(key);
  if (hit != ctx->plans.end()) return hit->second;
  MttkrpPlan p;
  auto t = ctx->tuned.find(key);
  if (t != ctx->tuned.end()) {
    p = mttkrp_plan(N, dims, n, R, fp32, t->second);
  } else {
    PlanOpts o{kTargetWgs, 0, 2, 4};
    const int cap = mttkrp_capacity(mttkrp_plan(N, dims, n, R, fp32, o), fp32);
    o.target_wgs = std::max(1, cap - 1);
    p = mttkrp_plan(N, dims, n, R, fp32, o);
  }
  return p;
}

// find_plan, remembered in the context's plan cache
MttkrpPlan get_plan(cp_ctx ctx, int N, const int64_t* dims, int n, int R, bool fp32) {
  const std::string key = plan_key(N, dims, n, R, fp32);
  auto hit = ctx->plans.find(key);
  if (hit != ctx->plans.end()) return hit->second;
  const MttkrpPlan p = find_plan(ctx, N, dims, n, R, fp32);
  ctx->plans[key] = p;
  return p;
}

// Launch plan of a sparse MTTKRP of mode n (not cached: it depends on nnz).
MttkrpPlan sparse_plan(const SpTensor& t, int n, int R) {
  MttkrpPlan p{};
  p.kind = kSparseKind;
  p.nsplit = sp_mttkrp_nsplit(t, n);
  p.partial_doubles = (size_t)p.nsplit * t.dims[n] * R;
  return p;
}

size_t max_partial(cp_ctx ctx, const int64_t* dims, int N, int R, bool fp32,
                   std::vector<MttkrpPlan>* plans, const SpTensor* sp = nullptr) {
  size_t mx = 0;
  for (int n = 0; n < N; ++n) {
    MttkrpPlan p = sp ? sparse_plan(*sp, n, R) : get_plan(ctx, N, dims, n, R, fp32);
    if (plans) plans->push_back(p);
    mx = std::max(mx, p.partial_doubles);
  }
  return mx;
}

int64_t max_dim(const int64_t* dims, int N) {
  int64_t m = 0;
  for (int i = 0; i < N; ++i) m = std::max(m, dims[i]);
  return m;
}

int64_t epi_blocks(int64_t In) { return (In + epi_rows_per_wg() - 1) / epi_rows_per_wg(); }

// Everything one BNGS/ALS sweep needs, carved from the workspace.
struct SweepWS {
  double* grams;
  double* sigma;
  double* partial;
  double* gram_part;
  double* scal_part;
  double* y;   // dimension tree: stage-1 tiles of the mode-1 launch (NULL: per-mode MTTKRPs)
};

template <typename Carver>
void carve_sweep(Carver& c, int N, int R, size_t partial, int64_t maxI, SweepWS* out,
                 size_t ydoubles = 0) {
  const int64_t nwg = epi_blocks(maxI);
  out->grams = c.template take<double>((size_t)N * R * R);
  out->sigma = c.template take<double>((size_t)N * R);
  out->partial = c.template take<double>(partial);
  out->gram_part = c.template take<double>((size_t)nwg * R * R);
  out->scal_part = c.template take<double>((size_t)std::max<int64_t>(nwg, 2048));
  out->y = ydoubles ? c.template take<double>(ydoubles) : nullptr;
}

// Launch plans of a sweep.  Dimension tree (order >= 3): the mode-1 launch runs
// its contraction unsplit and stores the stage-1 tiles
//   Y[s][i1][r] = sum_i0 Z(i0, i1, s) A^(0)(i0, r),
// which depend on Z and A^(0) only, so the MTTKRPs of modes >= 2 contract Y
// instead of streaming Z again: N - 1 passes over Z per sweep become 2.  Used
// when Y is at most a quarter of the tensor's bytes.
struct SweepPlan {
  std::vector<MttkrpPlan> p;   // per mode, direct MTTKRP
  bool dimtree = false;
  MttkrpPlan p1y{};            // mode 1 storing Y
  std::vector<int> ynsplit;    // modes >= 2 from Y
  size_t partial = 0;          // doubles of the partial-sum buffer
  size_t ydoubles = 0;
};

SweepPlan sweep_plan(cp_ctx ctx, const int64_t* dims, int N, int R, bool fp32,
                     const SpTensor* spt = nullptr) {
  SweepPlan sp;
  sp.partial = max_partial(ctx, dims, N, R, fp32, &sp.p, spt);
  if (!ctx->dimtree || N < 3 || spt) return sp;
  int64_t S = 1, P = 1;
  for (int m = 2; m < N; ++m) S *= dims[m];
  for (int m = 0; m < N; ++m) P *= dims[m];
  const size_t yd = (size_t)S * dims[1] * R;
  if (yd * 8 * 4 > (size_t)P * (fp32 ? 4 : 8)) return sp;
  // the tile-storing launch's own tuned options (cp_autotune times that
  // launch), else those of the plain mode-1 launch
  PlanOpts o = sp.p[1].opts;
  auto ty = ctx->tuned.find(plan_key(N, dims, 1, R, fp32) + ";y");
  if (ty != ctx->tuned.end()) o = ty->second;
  o.ksplit = 1;
  o.nostage = 0;   // the tile-storing variant runs with the factor staged
  const MttkrpPlan p1y = mttkrp_plan(N, dims, 1, R, fp32, o);
  if (p1y.ksplit != 1) return sp;   // Y needs the whole contraction in one piece
  sp.dimtree = true;
  sp.ydoubles = yd;
  sp.p1y = p1y;
  sp.partial = std::max(sp.partial, sp.p1y.partial_doubles);
  sp.ynsplit.assign(N, 0);
  for (int n = 2; n < N; ++n) {
    sp.ynsplit[n] = ymttkrp_nsplit(dims, N, n, R);
    sp.partial = std::max(sp.partial, (size_t)sp.ynsplit[n] * dims[n] * R);
  }
  return sp;
}

// Small-level relaxation (one workgroup, tensor in LDS) when the context allows
// it and the level fits; returns false when the general path must run.
bool try_small_relax(cp_ctx ctx, const int64_t* dims, int N, int R, const void* z, bool fp32,
                     double* const* A, float* const* A32, double* const* F, int gs_iters, int nsweeps,
                     cp_status* st) {
  if (!ctx->small || nsweeps <= 0) return false;
  SmallDesc d{};
  d.z = z;
  d.N = N;
  d.R = R;
  d.nsweeps = nsweeps;
  d.gs_iters = gs_iters;
  d.P = 1;
  for (int m = 0; m < N; ++m) {
    d.dims[m] = dims[m];
    d.P *= dims[m];
    d.A[m] = A[m];
    d.A32[m] = A32 ? A32[m] : nullptr;
    d.F[m] = F ? F[m] : nullptr;
  }
  if (!small_eligible(d, fp32)) return false;
  ProfScope ps(ctx, CP_PROF_OTHER);
  *st = hip_check(ctx, relax_small_launch(d, fp32, ctx->stream), "relax_small_launch");
  return true;
}

// `nsweeps` BNGS sweeps over all modes starting from the stored factors A.
// Enqueues: Grams of A, then per mode an MTTKRP launch (whose workgroup 0 does
// the sweep bookkeeping for the update) and the update, then one finalize.
cp_status enqueue_sweeps(cp_ctx ctx, const int64_t* dims, int N, int R, const void* z, bool fp32,
                         double* const* A, float* const* A32, double* const* F,
                         const SweepPlan& sp, const SweepWS& w, cp_solver solver,
                         int gs_iters, int normalize, int nsweeps, double* f_hist,
                         const double* norm2, const SpTensor* spt = nullptr) {
  if (nsweeps <= 0) return CP_OK;
  TRY(enqueue_gram(ctx, A, A32, dims, N, R, w.grams, w.sigma));
  auto base_args = [&](int n) {
    PrepArgs pa{};
    pa.N = N;
    pa.n = n;
    pa.R = R;
    pa.grams = w.grams;
    pa.sigma = w.sigma;
    pa.out = ctx->prep_out;
    pa.kind = ctx->chol_kind;
    pa.flags = ctx->flags;
    pa.solver = solver;
    pa.normalize = normalize;
    pa.norm2 = norm2;
    pa.inner_part = w.scal_part;
    pa.inner_count = (int32_t)epi_blocks(dims[N - 1]);
    return pa;
  };
  for (int k = 0; k < nsweeps; ++k) {
    for (int n = 0; n < N; ++n) {
      PrepArgs pa = base_args(n);
      if (k == 0 && n == 0) {
        pa.p = -1;
      } else {
        pa.p = (n + N - 1) % N;
        pa.Ap = A[pa.p];
        pa.Ip = dims[pa.p];
      }
      if (n == 0 && k > 0) {
        pa.boundary = 1;
        pa.f_slot = f_hist ? f_hist + (k - 1) : nullptr;
      }
      const bool tree = sp.dimtree && w.y;
      int nsplit = sp.p[n].nsplit;
      if (tree && n >= 2) {
        ProfScope ps(ctx, fp32 ? CP_PROF_MTTKRP_MODEN_F32 : CP_PROF_MTTKRP_MODEN_F64);
        HIPCHK(ymttkrp_launch(dims, N, n, R, w.y, fp32, (const double* const*)A, w.partial, sp.ynsplit[n],
                              &pa, ctx->stream));
        nsplit = sp.ynsplit[n];
      } else if (tree && n == 1) {
        ProfScope ps(ctx, fp32 ? CP_PROF_MTTKRP_MODE1_F32 : CP_PROF_MTTKRP_MODE1_F64);
        HIPCHK(mttkrp_launch(sp.p1y, dims, N, n, R, z, fp32, (const double* const*)A, (const float* const*)A32,
                             w.partial, &pa, ctx->stream, w.y));
        nsplit = sp.p1y.nsplit;
      } else {
        cp_status s = enqueue_mttkrp(ctx, dims, N, n, R, z, fp32, (const double* const*)A,
                                     (const float* const*)A32, sp.p[n], w.partial, &pa, spt);
        if (s != CP_OK) return s;
      }
      EpiDesc d{};
      d.op = EPI_UPDATE;
      d.solver = solver;
      d.gs_iters = gs_iters;
      d.R = R;
      d.N = N;
      d.n = n;
      d.nsplit = nsplit;
      d.In = dims[n];
      d.partial = w.partial;
      d.F = F ? F[n] : nullptr;
      d.A = A[n];
      d.A32 = A32 ? A32[n] : nullptr;
      d.grams = w.grams;
      d.prep_out = ctx->prep_out;
      d.kind = ctx->chol_kind;
      d.scal_part = w.scal_part;
      d.flags = ctx->flags;
      d.want_obj = (f_hist && n == N - 1) ? 1 : 0;
      TRY(enqueue_epi(ctx, d));
    }
  }
  PrepArgs fa = base_args(0);
  fa.p = N - 1;
  fa.Ap = A[N - 1];
  fa.Ip = dims[N - 1];
  fa.boundary = 1;
  fa.f_slot = f_hist ? f_hist + (nsweeps - 1) : nullptr;
  for (int m = 0; m < N; ++m) {
    fa.A[m] = A[m];
    fa.A32[m] = A32 ? A32[m] : nullptr;
    fa.dims[m] = dims[m];
  }
  ProfScope ps(ctx, CP_PROF_NORMALIZE);
  HIPCHK(finalize_launch(fa, ctx->stream));
  return CP_OK;
}


// One strided batched GEMM as launches that keep the grid's y and z extents
// within 65535 (column tiles of 64, batch entries).
cp_status gemm_chunked(cp_ctx ctx, const GemmDesc& g, bool fp32) {
  const int64_t esz = fp32 ? 4 : 8;
  const int64_t ncols = 65535LL * 64, nbat = 65535;
  for (int64_t b0 = 0; b0 < g.batch; b0 += nbat)
    for (int64_t n0 = 0; n0 < g.N; n0 += ncols) {
      GemmDesc h = g;
      h.batch = std::min(nbat, g.batch - b0);
      h.N = std::min(ncols, g.N - n0);
      h.A = (const char*)g.A + b0 * g.a_bs * esz;
      h.B = (const char*)g.B + (b0 * g.b_bs + n0 * g.b_cs) * esz;
      h.C = (char*)g.C + (b0 * g.c_bs + n0 * g.c_cs) * esz;
      HIPCHK(gemm_launch(h, fp32, ctx->stream));
    }
  return CP_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

cp_status cp_ctx_create(cp_ctx* out, void* hip_stream) {
  if (!out) return CP_ERR_INVALID;
  *out = nullptr;
  cp_ctx ctx = new (std::nothrow) cp_ctx_s();
  if (!ctx) return CP_ERR_NOMEM;
  ctx->stream = (hipStream_t)hip_stream;
  hipError_t e = hipGetDevice(&ctx->device);
  if (e != hipSuccess) {
    delete ctx;
    return CP_ERR_HIP;
  }
  e = scratch_lookup(ctx->device);
  if (e != hipSuccess) {
    delete ctx;
    return CP_ERR_HIP;
  }
  const size_t fixed_bytes = align_up(kNumCounters * sizeof(int32_t)) + align_up(64) +
                             align_up((kMaxRank * kMaxRank + 2 * kMaxRank) * sizeof(double)) +
                             align_up(64) +
                             align_up(64 * sizeof(double));
  e = hipMalloc((void**)&ctx->fixed, fixed_bytes);
  if (e != hipSuccess) {
    delete ctx;
    return CP_ERR_NOMEM;
  }
  e = hipMemset(ctx->fixed, 0, fixed_bytes);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(ctx->fixed);
    delete ctx;
    return CP_ERR_HIP;
  }
  Arena a(ctx->fixed);
  ctx->counters = a.take<int32_t>(kNumCounters);
  ctx->flags = a.take<uint32_t>(16);
  ctx->prep_out = a.take<double>(kMaxRank * kMaxRank + 2 * kMaxRank);
  ctx->chol_kind = a.take<int32_t>(16);
  ctx->scal = a.take<double>(64);
  *out = ctx;
  return CP_OK;
}

cp_status cp_ctx_destroy(cp_ctx ctx) {
  if (!ctx) return CP_ERR_INVALID;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& r : ctx->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  clear_graphs(ctx);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->fixed) (void)hipFree(ctx->fixed);
  delete ctx;
  return CP_OK;
}

cp_status cp_set_option(cp_ctx ctx, int32_t option, int32_t value) {
  if (!ctx) return CP_ERR_INVALID;
  if (option == CP_OPT_DIMTREE && (value == 0 || value == 1)) {
    ctx->dimtree = value;
    clear_graphs(ctx);
    return CP_OK;
  }
  if (option == CP_OPT_SMALL_LEVELS && (value == 0 || value == 1)) {
    ctx->small = value;
    clear_graphs(ctx);
    return CP_OK;
  }
  if (option == CP_OPT_GRAPHS && (value == 0 || value == 1)) {
    ctx->graphs = value;
    clear_graphs(ctx);
    return CP_OK;
  }
  return set_err(ctx, CP_ERR_INVALID, "cp_set_option: unknown option %d or value %d", option, value);
}

cp_status cp_set_stream(cp_ctx ctx, void* hip_stream) {
  if (!ctx) return CP_ERR_INVALID;
  ctx->stream = (hipStream_t)hip_stream;
  return CP_OK;
}

const char* cp_last_error(cp_ctx ctx) { return ctx ? ctx->err.c_str() : "invalid context"; }

cp_status cp_get_status(cp_ctx ctx, int32_t* flags) {
  if (!ctx) return CP_ERR_INVALID;
  if (!flags) return set_err(ctx, CP_ERR_INVALID, "flags is NULL");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  uint32_t h = 0;
  HIPCHK(hipMemcpy(&h, ctx->flags, sizeof(h), hipMemcpyDeviceToHost));
  HIPCHK(hipMemset(ctx->flags, 0, sizeof(uint32_t)));
  HIPCHK(hipDeviceSynchronize());
  *flags = (int32_t)h;
  return CP_OK;
}

cp_status cp_cast_f32(cp_ctx ctx, const double* src, float* dst, int64_t count) {
  if (!ctx) return CP_ERR_INVALID;
  if (!src || !dst) return set_err(ctx, CP_ERR_INVALID, "cp_cast_f32: NULL pointer");
  if (count < 0) return set_err(ctx, CP_ERR_SHAPE, "cp_cast_f32: negative count");
  if (count == 0) return CP_OK;
  HIPCHK(cast_launch(src, dst, count, ctx->stream));
  return CP_OK;
}

cp_status cp_norm2(cp_ctx ctx, const cp_tensor* Z, double* out) {
  if (!ctx) return CP_ERR_INVALID;
  cp_status s = check_tensor(ctx, Z, true, false, "Z");
  if (s != CP_OK) return s;
  if (!out) return set_err(ctx, CP_ERR_INVALID, "cp_norm2: out is NULL");
  s = ensure_ws(ctx, align_up(2048 * sizeof(double)));
  if (s != CP_OK) return s;
  if (is_sparse(Z))
    HIPCHK(norm2_launch(Z->vals, Z->nnz, (double*)ctx->ws, ctx->counters + CNT_DOT, out, ctx->stream));
  else
    HIPCHK(norm2_launch(Z->z64, numel(Z), (double*)ctx->ws, ctx->counters + CNT_DOT, out, ctx->stream));
  return CP_OK;
}

cp_status cp_sparse_index(cp_ctx ctx, int32_t order, const int64_t* dims, int64_t nnz,
                          const int32_t* idx, int64_t* rowptr, int32_t* perm) {
  if (!dims || !idx || !rowptr || !perm)
    return ctx ? set_err(ctx, CP_ERR_INVALID, "cp_sparse_index: NULL pointer") : CP_ERR_INVALID;
  std::string msg;
  const cp_status s = sparse_index_host(order, dims, nnz, idx, rowptr, perm, &msg);
  if (s != CP_OK && ctx) return set_err(ctx, s, "cp_sparse_index: %s", msg.c_str());
  return s;
}

cp_status cp_mttkrp(cp_ctx ctx, const cp_tensor* Z, const cp_factors* A, int32_t n, double* M,
                    cp_prec prec) {
  if (!ctx) return CP_ERR_INVALID;
  cp_status s = check_prec(ctx, prec);
  if (s != CP_OK) return s;
  const bool mixed = prec == CP_MIXED;
  if ((s = check_tensor(ctx, Z, !mixed, mixed, "Z")) != CP_OK) return s;
  const int N = Z->order;
  if ((s = check_factors(ctx, A, N, mixed, "A")) != CP_OK) return s;
  if (n < 0 || n >= N) return set_err(ctx, CP_ERR_INVALID, "cp_mttkrp: mode %d outside [0, %d)", n, N);
  if (!M) return set_err(ctx, CP_ERR_INVALID, "cp_mttkrp: M is NULL");
  const int R = A->rank;
  const SpTensor spv = is_sparse(Z) ? sp_view(Z) : SpTensor{};
  const SpTensor* spt = is_sparse(Z) ? &spv : nullptr;
  MttkrpPlan plan = spt ? sparse_plan(spv, n, R) : get_plan(ctx, N, Z->dims, n, R, mixed);
  const void* z = mixed ? (const void*)Z->z32 : (const void*)Z->z64;
  if (plan.nsplit == 1)
    return enqueue_mttkrp(ctx, Z->dims, N, n, R, z, mixed, A->a, (const float* const*)A->a32, plan, M,
                          nullptr, spt);
  if ((s = ensure_ws(ctx, align_up(plan.partial_doubles * sizeof(double)))) != CP_OK) return s;
  double* part = (double*)ctx->ws;
  if ((s = enqueue_mttkrp(ctx, Z->dims, N, n, R, z, mixed, A->a, (const float* const*)A->a32, plan,
                          part, nullptr, spt)) != CP_OK)
    return s;
  EpiDesc d{};
  d.op = EPI_STORE_M;
  d.R = R;
  d.N = N;
  d.n = n;
  d.nsplit = plan.nsplit;
  d.In = Z->dims[n];
  d.partial = part;
  d.outbuf = M;
  TRY(enqueue_epi(ctx, d));
  return CP_OK;
}

cp_status cp_mttkrp_noalloc(cp_ctx ctx, const cp_tensor* Z, const cp_factors* A, int32_t n,
                            double* M, cp_prec prec) {
  if (!ctx) return CP_ERR_INVALID;
  cp_status s = check_prec(ctx, prec);
  if (s != CP_OK) return s;
  const bool mixed = prec == CP_MIXED;
  if ((s = check_tensor(ctx, Z, !mixed, mixed, "Z")) != CP_OK) return s;
  if ((s = require_dense(ctx, Z, "cp_mttkrp_noalloc")) != CP_OK) return s;
  const int N = Z->order;
  if ((s = check_factors(ctx, A, N, mixed, "A")) != CP_OK) return s;
  if (n < 0 || n >= N) return set_err(ctx, CP_ERR_INVALID, "cp_mttkrp_noalloc: mode %d outside [0, %d)", n, N);
  if (!M) return set_err(ctx, CP_ERR_INVALID, "cp_mttkrp_noalloc: M is NULL");
  int device = -1;
  HIPCHK(hipGetDevice(&device));
  if (device < 0 || device >= kMaxDevices || !g_scratch[device])
    return set_err(ctx, CP_ERR_HIP, "cp_mttkrp_noalloc: no scratch address for device %d "
                   "(create a context on that device first)", device);
  const int R = A->rank;
  // the launch configuration cp_mttkrp uses, without adding it to the plan cache
  const MttkrpPlan plan = find_plan(ctx, N, Z->dims, n, R, mixed);
  const void* z = mixed ? (const void*)Z->z32 : (const void*)Z->z64;
  if (plan.nsplit == 1)
    return enqueue_mttkrp(ctx, Z->dims, N, n, R, z, mixed, A->a, (const float* const*)A->a32, plan, M);
  const size_t need = plan.partial_doubles * sizeof(double);
  if (need > (size_t)CP_NOALLOC_SCRATCH_BYTES)
    return set_err(ctx, CP_ERR_SHAPE,
                   "cp_mttkrp_noalloc: mode %d needs %zu bytes of partial sums, the static scratch "
                   "holds %zu (use cp_mttkrp)", n, need, (size_t)CP_NOALLOC_SCRATCH_BYTES);
  double* part = (double*)g_scratch[device];
  if ((s = enqueue_mttkrp(ctx, Z->dims, N, n, R, z, mixed, A->a, (const float* const*)A->a32, plan,
                          part)) != CP_OK)
    return s;
  EpiDesc d{};
  d.op = EPI_STORE_M;
  d.R = R;
  d.N = N;
  d.n = n;
  d.nsplit = plan.nsplit;
  d.In = Z->dims[n];
  d.partial = part;
  d.outbuf = M;
  TRY(enqueue_epi(ctx, d));
  return CP_OK;
}

cp_status cp_als_sweep(cp_ctx ctx, const cp_tensor* Z, cp_factors* A, const cp_factors* F,
                       int32_t nsweeps, cp_solver solver, int32_t gs_iters, int32_t normalize,
                       cp_prec prec, double* f_hist) {
  if (!ctx) return CP_ERR_INVALID;
  cp_status s = check_prec(ctx, prec);
  if (s != CP_OK) return s;
  const bool mixed = prec == CP_MIXED;
  if ((s = check_tensor(ctx, Z, !mixed, mixed, "Z")) != CP_OK) return s;
  const int N = Z->order;
  if ((s = check_factors(ctx, A, N, mixed, "A")) != CP_OK) return s;
  if (F) {
    for (int m = 0; m < N; ++m)
      if (!F->a[m]) return set_err(ctx, CP_ERR_INVALID, "F->a[%d] is NULL", m);
  }
  if (nsweeps < 0) return set_err(ctx, CP_ERR_INVALID, "nsweeps < 0");
  if (solver != CP_SOLVE_CHOL && solver != CP_SOLVE_GS)
    return set_err(ctx, CP_ERR_INVALID, "unknown solver %d", (int)solver);
  if (solver == CP_SOLVE_GS && (gs_iters < 1 || gs_iters > 1000))
    return set_err(ctx, CP_ERR_INVALID, "gs_iters %d outside [1, 1000]", gs_iters);
  if (f_hist && !Z->norm2) return set_err(ctx, CP_ERR_INVALID, "f_hist needs Z->norm2");
  if (nsweeps == 0) return CP_OK;
  const int R = A->rank;
  const SpTensor spv = is_sparse(Z) ? sp_view(Z) : SpTensor{};
  const SpTensor* spt = is_sparse(Z) ? &spv : nullptr;
  {
    bool h32 = true;
    for (int m = 0; m < N; ++m) h32 = h32 && A->a32[m];
    cp_status st = CP_OK;
    if (solver == CP_SOLVE_GS && !normalize && !f_hist && !spt &&
        try_small_relax(ctx, Z->dims, N, R, mixed ? (const void*)Z->z32 : (const void*)Z->z64, mixed, A->a,
                        h32 ? A->a32 : nullptr, F ? F->a : nullptr, gs_iters, nsweeps, &st))
      return st;
  }
  const SweepPlan sp = sweep_plan(ctx, Z->dims, N, R, mixed, spt);
  Sizer sz;
  SweepWS w{};
  carve_sweep(sz, N, R, sp.partial, max_dim(Z->dims, N), &w, sp.ydoubles);
  if ((s = ensure_ws(ctx, sz.off)) != CP_OK) return s;
  Arena ar(ctx->ws);
  carve_sweep(ar, N, R, sp.partial, max_dim(Z->dims, N), &w, sp.ydoubles);
  bool have32 = true;
  for (int m = 0; m < N; ++m) have32 = have32 && A->a32[m];
  const void* z = mixed ? (const void*)Z->z32 : (const void*)Z->z64;
  return enqueue_sweeps(ctx, Z->dims, N, R, z, mixed, A->a, have32 ? A->a32 : nullptr,
                        F ? F->a : nullptr, sp, w, solver, gs_iters, normalize, nsweeps, f_hist,
                        Z->norm2, spt);
}

cp_status cp_objective(cp_ctx ctx, const cp_tensor* Z, const cp_factors* A, int32_t exact,
                       double* f, double* g, cp_prec prec) {
  if (!ctx) return CP_ERR_INVALID;
  cp_status s = check_prec(ctx, prec);
  if (s != CP_OK) return s;
  const bool mixed = prec == CP_MIXED;
  const bool need64 = (f && exact) || !mixed;
  if ((s = check_tensor(ctx, Z, need64, mixed && (g || (f && !exact)), "Z")) != CP_OK) return s;
  const int N = Z->order;
  if ((s = check_factors(ctx, A, N, mixed && (g || (f && !exact)), "A")) != CP_OK) return s;
  if (!f && !g) return CP_OK;
  const SpTensor spv = is_sparse(Z) ? sp_view(Z) : SpTensor{};
  const SpTensor* spt = is_sparse(Z) ? &spv : nullptr;
  if (spt) exact = 0;   // the sparse form has no residual pass: fused identity
  if ((g || (f && !exact)) && !Z->norm2)
    return set_err(ctx, CP_ERR_INVALID, "cp_objective: g and the fused f need Z->norm2");
  const int R = A->rank;
  std::vector<MttkrpPlan> plans;
  const size_t part = max_partial(ctx, Z->dims, N, R, mixed, &plans, spt);
  const int64_t In_last = Z->dims[N - 1];
  Sizer sz;
  SweepWS w{};
  carve_sweep(sz, N, R, part, max_dim(Z->dims, N), &w);
  sz.take<double>((size_t)In_last * R);
  if ((s = ensure_ws(ctx, sz.off)) != CP_OK) return s;
  Arena ar(ctx->ws);
  carve_sweep(ar, N, R, part, max_dim(Z->dims, N), &w);
  double* Mlast = ar.take<double>((size_t)In_last * R);
  const void* z = mixed ? (const void*)Z->z32 : (const void*)Z->z64;
  if (f && exact)
    HIPCHK(residual_launch(Z->z64, Z->dims, N, R, A->a, w.scal_part, ctx->counters + CNT_RES, f,
                           ctx->stream));
  if (g || (f && !exact)) TRY(enqueue_gram(ctx, A->a, nullptr, Z->dims, N, R, w.grams));
  if (g) {
    for (int n = 0; n < N; ++n) {
      if ((s = enqueue_mttkrp(ctx, Z->dims, N, n, R, z, mixed, A->a, (const float* const*)A->a32,
                              plans[n], w.partial, nullptr, spt)) != CP_OK)
        return s;
      EpiDesc d{};
      d.op = EPI_GRAD;
      d.R = R;
      d.N = N;
      d.n = n;
      d.nsplit = plans[n].nsplit;
      d.In = Z->dims[n];
      d.partial = w.partial;
      d.A = A->a[n];
      d.grams = w.grams;
      d.scal_part = w.scal_part;
      d.counter = ctx->counters + CNT_EPI;
      d.scalar_out = ctx->scal;
      d.accumulate = n > 0;
      TRY(enqueue_epi(ctx, d));
    }
    HIPCHK(finish_g_launch(ctx->scal, Z->norm2, g, ctx->stream));
  }
  if (f && !exact) {
    if ((s = enqueue_mttkrp(ctx, Z->dims, N, N - 1, R, z, mixed, A->a, (const float* const*)A->a32,
                            plans[N - 1], w.partial, nullptr, spt)) != CP_OK)
      return s;
    EpiDesc d{};
    d.op = EPI_STORE_M;
    d.R = R;
    d.N = N;
    d.n = N - 1;
    d.nsplit = plans[N - 1].nsplit;
    d.In = In_last;
    d.partial = w.partial;
    d.outbuf = Mlast;
    TRY(enqueue_epi(ctx, d));
    HIPCHK(inner_launch(A->a[N - 1], Mlast, In_last * R, w.gram_part, ctx->counters + CNT_DOT,
                        ctx->scal + 1, ctx->stream));
    HIPCHK(fused_f_launch(w.grams, N, R, ctx->scal + 1, Z->norm2, f, ctx->stream));
  }
  return CP_OK;
}

cp_status cp_restrict(cp_ctx ctx, const cp_tensor* Z, const double* const phat[CP_MAX_ORDER],
                      cp_tensor* Zc, cp_prec prec) {
  if (!ctx) return CP_ERR_INVALID;
  cp_status s = check_prec(ctx, prec);
  if (s != CP_OK) return s;
  const bool mixed = prec == CP_MIXED;
  if ((s = check_tensor(ctx, Z, !mixed, mixed, "Z")) != CP_OK) return s;
  if (!Zc) return set_err(ctx, CP_ERR_INVALID, "Zc is NULL");
  if (!phat) return set_err(ctx, CP_ERR_INVALID, "phat array is NULL");
  const int N = Z->order;
  if (Zc->order != N) return set_err(ctx, CP_ERR_SHAPE, "Zc order %d != %d", Zc->order, N);
  if (mixed ? !Zc->z32 : !Zc->z64) return set_err(ctx, CP_ERR_INVALID, "Zc has no output buffer for this precision");
  if (Zc->nnz != 0) return set_err(ctx, CP_ERR_INVALID, "Zc must be in the dense form");
  int64_t dc[CP_MAX_ORDER];
  std::vector<int> modes;
  for (int m = 0; m < N; ++m) {
    dc[m] = phat[m] ? (Z->dims[m] + 1) / 2 : Z->dims[m];
    if (Zc->dims[m] != dc[m])
      return set_err(ctx, CP_ERR_SHAPE, "Zc->dims[%d] = %lld, expected %lld", m,
                     (long long)Zc->dims[m], (long long)dc[m]);
    if (phat[m]) modes.push_back(m);
  }
  const size_t esz = mixed ? 4 : 8;
  const void* src = mixed ? (const void*)Z->z32 : (const void*)Z->z64;
  void* dst = mixed ? (void*)Zc->z32 : (void*)Zc->z64;
  const int64_t P = numel(Z);
  const bool sparse = is_sparse(Z);
  if (modes.empty()) {
    if (sparse) {
      HIPCHK(fill_launch((double*)dst, 0.0, P, ctx->stream));
      HIPCHK(sp_densify_launch(sp_view(Z), (double*)dst, ctx->stream));
    } else {
      HIPCHK(hipMemcpyAsync(dst, src, P * esz, hipMemcpyDeviceToDevice, ctx->stream));
    }
    return CP_OK;
  }
  // intermediate sizes: after each restricted mode
  int64_t cur[CP_MAX_ORDER];
  for (int m = 0; m < N; ++m) cur[m] = Z->dims[m];
  size_t maxmid = 0;
  for (size_t q = 0; q + 1 < modes.size(); ++q) {
    cur[modes[q]] = dc[modes[q]];
    int64_t p = 1;
    for (int m = 0; m < N; ++m) p *= cur[m];
    maxmid = std::max(maxmid, (size_t)p);
  }
  Sizer sz;
  if (sparse) sz.take<double>((size_t)P);
  sz.take<char>(maxmid * esz);
  sz.take<char>(maxmid * esz);
  if (mixed)
    for (int m : modes) sz.take<float>((size_t)Z->dims[m] * dc[m]);
  if ((s = ensure_ws(ctx, sz.off)) != CP_OK) return s;
  Arena ar(ctx->ws);
  double* dense = sparse ? ar.take<double>((size_t)P) : nullptr;
  char* buf[2] = {ar.take<char>(maxmid * esz), ar.take<char>(maxmid * esz)};
  const void* pmat[CP_MAX_ORDER] = {};
  for (int m : modes) {
    if (mixed) {
      float* p32 = ar.take<float>((size_t)Z->dims[m] * dc[m]);
      HIPCHK(cast_launch(phat[m], p32, Z->dims[m] * dc[m], ctx->stream));
      pmat[m] = p32;
    } else {
      pmat[m] = phat[m];
    }
  }
  if (sparse) {
    // the entries scattered into a dense copy; the mode products below make
    // the coarse tensor dense whatever the input's sparsity
    HIPCHK(fill_launch(dense, 0.0, P, ctx->stream));
    HIPCHK(sp_densify_launch(sp_view(Z), dense, ctx->stream));
    src = dense;
  }
  for (int m = 0; m < N; ++m) cur[m] = Z->dims[m];
  const void* in = src;
  for (size_t q = 0; q < modes.size(); ++q) {
    const int n = modes[q];
    void* outp = (q + 1 == modes.size()) ? dst : (void*)buf[q & 1];
    int64_t L = 1, T = 1;
    for (int m = 0; m < n; ++m) L *= cur[m];
    for (int m = n + 1; m < N; ++m) T *= cur[m];
    const int64_t In = cur[n], Ic = dc[n];
    GemmDesc g{};
    if (n == 0) {
      // C (Ic x T) = P^^T (Ic x In) * X (In x T)
      g.A = pmat[n]; g.B = in; g.C = outp;
      g.M = Ic; g.N = T; g.K = In; g.batch = 1;
      g.a_rs = 1; g.a_cs = Ic; g.a_bs = 0;
      g.b_rs = 1; g.b_cs = In; g.b_bs = 0;
      g.c_rs = 1; g.c_cs = Ic; g.c_bs = 0;
    } else if (L >= 16 || L >= T) {
      // per t: C_t (L x Ic) = X_t (L x In) * P^ (In x Ic)
      g.A = in; g.B = pmat[n]; g.C = outp;
      g.M = L; g.N = Ic; g.K = In; g.batch = T;
      g.a_rs = 1; g.a_cs = L; g.a_bs = L * In;
      g.b_rs = Ic; g.b_cs = 1; g.b_bs = 0;
      g.c_rs = 1; g.c_cs = L; g.c_bs = L * Ic;
    } else {
      // few leading entries: per l, C_l (Ic x T) = P^^T (Ic x In) * X_l (In x T)
      // with X_l(k, t) = X[l + L k + L In t] (fills the 64-row tiles)
      g.A = pmat[n]; g.B = in; g.C = outp;
      g.M = Ic; g.N = T; g.K = In; g.batch = L;
      g.a_rs = 1; g.a_cs = Ic; g.a_bs = 0;
      g.b_rs = L; g.b_cs = L * In; g.b_bs = 1;
      g.c_rs = L; g.c_cs = L * Ic; g.c_bs = 1;
    }
    TRY(gemm_chunked(ctx, g, mixed));
    cur[n] = Ic;
    in = outp;
  }
  return CP_OK;
}

cp_status cp_restrict_factored(cp_ctx ctx, const cp_tensor* Z, const double* const w[CP_MAX_ORDER],
                               cp_tensor* Zc, cp_prec prec) {
  if (!ctx) return CP_ERR_INVALID;
  cp_status s = check_prec(ctx, prec);
  if (s != CP_OK) return s;
  const bool mixed = prec == CP_MIXED;
  if ((s = check_tensor(ctx, Z, !mixed, mixed, "Z")) != CP_OK) return s;
  if (!Zc) return set_err(ctx, CP_ERR_INVALID, "Zc is NULL");
  if (!w) return set_err(ctx, CP_ERR_INVALID, "weights array is NULL");
  const int N = Z->order;
  if (Zc->order != N) return set_err(ctx, CP_ERR_SHAPE, "Zc order %d != %d", Zc->order, N);
  if (mixed ? !Zc->z32 : !Zc->z64) return set_err(ctx, CP_ERR_INVALID, "Zc has no output buffer for this precision");
  if (Zc->nnz != 0) return set_err(ctx, CP_ERR_INVALID, "Zc must be in the dense form");
  int64_t dc[CP_MAX_ORDER];
  std::vector<int> modes;
  for (int m = 0; m < N; ++m) {
    if (w[m] && Z->dims[m] < 2)
      return set_err(ctx, CP_ERR_SHAPE, "mode %d: extent %lld cannot be coarsened", m, (long long)Z->dims[m]);
    dc[m] = w[m] ? (Z->dims[m] + 1) / 2 : Z->dims[m];
    if (Zc->dims[m] != dc[m])
      return set_err(ctx, CP_ERR_SHAPE, "Zc->dims[%d] = %lld, expected %lld", m,
                     (long long)Zc->dims[m], (long long)dc[m]);
    if (w[m]) modes.push_back(m);
  }
  const size_t esz = mixed ? 4 : 8;
  const void* src = mixed ? (const void*)Z->z32 : (const void*)Z->z64;
  void* dst = mixed ? (void*)Zc->z32 : (void*)Zc->z64;
  const int64_t P = numel(Z);
  const bool sparse = is_sparse(Z);
  if (modes.empty()) {
    if (sparse) {
      HIPCHK(fill_launch((double*)dst, 0.0, P, ctx->stream));
      HIPCHK(sp_densify_launch(sp_view(Z), (double*)dst, ctx->stream));
    } else {
      HIPCHK(hipMemcpyAsync(dst, src, P * esz, hipMemcpyDeviceToDevice, ctx->stream));
    }
    return CP_OK;
  }
  int64_t cur[CP_MAX_ORDER];
  for (int m = 0; m < N; ++m) cur[m] = Z->dims[m];
  size_t maxmid = 0;
  for (size_t q = 0; q + 1 < modes.size(); ++q) {
    cur[modes[q]] = dc[modes[q]];
    int64_t p = 1;
    for (int m = 0; m < N; ++m) p *= cur[m];
    maxmid = std::max(maxmid, (size_t)p);
  }
  Sizer sz;
  if (sparse) sz.take<double>((size_t)P);
  sz.take<char>(maxmid * esz);
  sz.take<char>(maxmid * esz);
  for (int m : modes) sz.take<double>((size_t)6 * dc[m]);
  if ((s = ensure_ws(ctx, sz.off)) != CP_OK) return s;
  Arena ar(ctx->ws);
  double* dense = sparse ? ar.take<double>((size_t)P) : nullptr;
  char* buf[2] = {ar.take<char>(maxmid * esz), ar.take<char>(maxmid * esz)};
  double* coef[CP_MAX_ORDER] = {};
  RCoefJobs jobs{};
  for (int m : modes) {
    coef[m] = ar.take<double>((size_t)6 * dc[m]);   // 4 Ic coefficients + 2 Ic scratch
    const int q = jobs.count++;
    jobs.I[q] = Z->dims[m];
    jobs.w[q] = w[m];
    jobs.coef[q] = coef[m];
    jobs.scratch[q] = coef[m] + 4 * dc[m];
  }
  HIPCHK(restrict_coef_launch(jobs, ctx->stream));
  if (sparse) {
    HIPCHK(fill_launch(dense, 0.0, P, ctx->stream));
    HIPCHK(sp_densify_launch(sp_view(Z), dense, ctx->stream));
    src = dense;
  }
  for (int m = 0; m < N; ++m) cur[m] = Z->dims[m];
  const void* in = src;
  for (size_t q = 0; q < modes.size(); ++q) {
    const int n = modes[q];
    void* outp = (q + 1 == modes.size()) ? dst : (void*)buf[q & 1];
    int64_t L = 1, T = 1;
    for (int m = 0; m < n; ++m) L *= cur[m];
    for (int m = n + 1; m < N; ++m) T *= cur[m];
    HIPCHK(restrict_factored_launch(in, outp, L, cur[n], T, coef[n], mixed, ctx->stream));
    cur[n] = dc[n];
    in = outp;
  }
  return CP_OK;
}

cp_status cp_prolong(cp_ctx ctx, int64_t I, int64_t Ic, int32_t R, const double* phat,
                     const double* Ac, const double* Ac_tilde, double* A) {
  if (!ctx) return CP_ERR_INVALID;
  if (!Ac || !A) return set_err(ctx, CP_ERR_INVALID, "cp_prolong: NULL pointer");
  if (I < 1 || Ic < 1 || R < 1 || R > CP_MAX_RANK) return set_err(ctx, CP_ERR_SHAPE, "cp_prolong: bad sizes");
  if (!phat && Ic != I) return set_err(ctx, CP_ERR_SHAPE, "cp_prolong: identity transfer needs Ic == I");
  HIPCHK(prolong_launch(I, Ic, R, phat, Ac, Ac_tilde, A, ctx->stream));
  return CP_OK;
}

cp_status cp_restrict_factor(cp_ctx ctx, int64_t I, int64_t Ic, int32_t R, const double* phat,
                             const double* A, double* Ac) {
  if (!ctx) return CP_ERR_INVALID;
  if (!A || !Ac) return set_err(ctx, CP_ERR_INVALID, "cp_restrict_factor: NULL pointer");
  if (I < 1 || Ic < 1 || R < 1 || R > CP_MAX_RANK) return set_err(ctx, CP_ERR_SHAPE, "cp_restrict_factor: bad sizes");
  if (!phat && Ic != I) return set_err(ctx, CP_ERR_SHAPE, "cp_restrict_factor: identity transfer needs Ic == I");
  HIPCHK(restrict_factor_launch(I, Ic, R, phat, A, Ac, ctx->stream));
  return CP_OK;
}

cp_status cp_interp_weights(cp_ctx ctx, const cp_tensor* Z, const cp_factors* A, int32_t groups,
                            int32_t nfit, int32_t n, double* w) {
  if (!ctx) return CP_ERR_INVALID;
  cp_status s = check_tensor(ctx, Z, true, false, "Z");
  if (s != CP_OK) return s;
  const int N = Z->order;
  if ((s = check_factors(ctx, A, N, false, "A")) != CP_OK) return s;
  if (groups < 1 || groups > kMaxGroups || A->rank % groups != 0)
    return set_err(ctx, CP_ERR_INVALID, "cp_interp_weights: %d groups do not split rank %d (at most %d groups)",
                   groups, A->rank, kMaxGroups);
  if (nfit < 1 || nfit > groups)
    return set_err(ctx, CP_ERR_INVALID, "cp_interp_weights: nfit %d outside [1, %d]", nfit, groups);
  if (n < 0 || n >= N) return set_err(ctx, CP_ERR_INVALID, "cp_interp_weights: mode %d outside [0, %d)", n, N);
  if (Z->dims[n] < 2) return set_err(ctx, CP_ERR_SHAPE, "cp_interp_weights: mode %d has extent < 2", n);
  if (!w) return set_err(ctx, CP_ERR_INVALID, "cp_interp_weights: w is NULL");
  const int Rt = A->rank;
  const int64_t In = Z->dims[n];
  const SpTensor spv = is_sparse(Z) ? sp_view(Z) : SpTensor{};
  const SpTensor* spt = is_sparse(Z) ? &spv : nullptr;
  const MttkrpPlan plan = spt ? sparse_plan(spv, n, Rt) : get_plan(ctx, N, Z->dims, n, Rt, false);
  Sizer sz;
  sz.take<double>((size_t)N * Rt * Rt);
  sz.take<double>((size_t)In * Rt);
  sz.take<double>(plan.partial_doubles);
  if ((s = ensure_ws(ctx, sz.off)) != CP_OK) return s;
  Arena ar(ctx->ws);
  double* grams = ar.take<double>((size_t)N * Rt * Rt);
  double* M = ar.take<double>((size_t)In * Rt);
  double* part = ar.take<double>(plan.partial_doubles);
  TRY(enqueue_gram(ctx, A->a, nullptr, Z->dims, N, Rt, grams));
  if (plan.nsplit == 1) {
    TRY(enqueue_mttkrp(ctx, Z->dims, N, n, Rt, Z->z64, false, A->a, nullptr, plan, M, nullptr, spt));
  } else {
    TRY(enqueue_mttkrp(ctx, Z->dims, N, n, Rt, Z->z64, false, A->a, nullptr, plan, part, nullptr, spt));
    EpiDesc d{};
    d.op = EPI_STORE_M;
    d.R = Rt;
    d.N = N;
    d.n = n;
    d.nsplit = plan.nsplit;
    d.In = In;
    d.partial = part;
    d.outbuf = M;
    TRY(enqueue_epi(ctx, d));
  }
  ProfScope ps(ctx, CP_PROF_OTHER);
  HIPCHK(interp_weights_launch(A->a[n], M, grams, N, n, In, Rt, Rt / groups, nfit, w, ctx->stream));
  return CP_OK;
}

cp_status cp_transfer_build(cp_ctx ctx, int64_t I, const double* w, double* phat) {
  if (!ctx) return CP_ERR_INVALID;
  if (!w || !phat) return set_err(ctx, CP_ERR_INVALID, "cp_transfer_build: NULL pointer");
  if (I < 2) return set_err(ctx, CP_ERR_SHAPE, "cp_transfer_build: I = %lld < 2", (long long)I);
  const int64_t Ic = (I + 1) / 2;
  cp_status s = ensure_ws(ctx, align_up(2 * Ic * sizeof(double)));
  if (s != CP_OK) return s;
  HIPCHK(transfer_build_launch(I, w, phat, (double*)ctx->ws, ctx->stream));
  return CP_OK;
}

// The bookkeeping workgroup of mode n's launch inside an ALS sweep (the sweep
// boundary falls on mode 0), on scratch Grams and column scales: timed launches
// then have the same configuration and work as the launches of a sweep.  It
// writes only the scratch arrays and the context's own prep/flag words.
static PrepArgs timing_prep(cp_ctx ctx, const cp_tensor* Z, const cp_factors* A, int n,
                            double* grams, double* sigma) {
  const int N = Z->order;
  PrepArgs pa{};
  pa.N = N;
  pa.n = n;
  pa.R = A->rank;
  pa.grams = grams;
  pa.sigma = sigma;
  pa.out = ctx->prep_out;
  pa.kind = ctx->chol_kind;
  pa.flags = ctx->flags;
  pa.solver = CP_SOLVE_CHOL;
  pa.p = (n + N - 1) % N;
  pa.Ap = A->a[pa.p];
  pa.Ip = Z->dims[pa.p];
  pa.boundary = n == 0;
  pa.normalize = 1;
  return pa;
}

cp_status cp_time_mttkrp(cp_ctx ctx, const cp_tensor* Z, const cp_factors* A, int32_t n,
                         cp_prec prec, int32_t reps, double* ms) {
  if (!ctx) return CP_ERR_INVALID;
  cp_status s = check_prec(ctx, prec);
  if (s != CP_OK) return s;
  const bool mixed = prec == CP_MIXED;
  if ((s = check_tensor(ctx, Z, !mixed, mixed, "Z")) != CP_OK) return s;
  if ((s = require_dense(ctx, Z, "timing and tuning calls")) != CP_OK) return s;
  const int N = Z->order;
  if ((s = check_factors(ctx, A, N, mixed, "A")) != CP_OK) return s;
  if (n < 0 || n >= N) return set_err(ctx, CP_ERR_INVALID, "cp_time_mttkrp: bad mode %d", n);
  if (reps < 1 || !ms) return set_err(ctx, CP_ERR_INVALID, "cp_time_mttkrp: reps < 1 or ms NULL");
  const int R = A->rank;
  // the launch the sweep makes for mode n: with the dimension tree, mode 1 also
  // stores Y and modes >= 2 contract Y (filled by one untimed mode-1 launch)
  const SweepPlan sp = sweep_plan(ctx, Z->dims, N, R, mixed);
  const bool tree = sp.dimtree && n >= 1;
  const MttkrpPlan plan = tree ? sp.p1y : get_plan(ctx, N, Z->dims, n, R, mixed);
  Sizer sz;
  sz.take<double>((size_t)N * R * R);
  sz.take<double>((size_t)N * R);
  sz.take<double>(tree ? sp.partial : plan.partial_doubles);
  sz.take<double>(tree ? sp.ydoubles : 0);
  if ((s = ensure_ws(ctx, sz.off)) != CP_OK) return s;
  Arena ar(ctx->ws);
  double* grams = ar.take<double>((size_t)N * R * R);
  double* sigma = ar.take<double>((size_t)N * R);
  double* part = ar.take<double>(tree ? sp.partial : plan.partial_doubles);
  double* y = tree ? ar.take<double>(sp.ydoubles) : nullptr;
  HIPCHK(gram_launch(A->a, nullptr, Z->dims, N, R, grams, ctx->stream, sigma));
  const PrepArgs pa = timing_prep(ctx, Z, A, n, grams, sigma);
  const void* z = mixed ? (const void*)Z->z32 : (const void*)Z->z64;
  auto launch = [&]() -> hipError_t {
    if (tree && n >= 2)
      return ymttkrp_launch(Z->dims, N, n, R, y, mixed, A->a, part, sp.ynsplit[n], &pa, ctx->stream);
    return mttkrp_launch(plan, Z->dims, N, n, R, z, mixed, A->a, (const float* const*)A->a32, part, &pa,
                         ctx->stream, y);
  };
  if (tree && n >= 2) {
    const PrepArgs pa1 = timing_prep(ctx, Z, A, 1, grams, sigma);
    HIPCHK(mttkrp_launch(sp.p1y, Z->dims, N, 1, R, z, mixed, A->a, (const float* const*)A->a32, part, &pa1,
                         ctx->stream, y));
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, ctx->stream));
  for (int k = 0; k < reps; ++k) HIPCHK(launch());
  HIPCHK(hipEventRecord(e1, ctx->stream));
  HIPCHK(hipEventSynchronize(e1));
  float t = 0.f;
  HIPCHK(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = (double)t / reps;
  return CP_OK;
}

cp_status cp_autotune(cp_ctx ctx, const cp_tensor* Z, const cp_factors* A, cp_prec prec,
                      int32_t reps) {
  if (!ctx) return CP_ERR_INVALID;
  cp_status s = check_prec(ctx, prec);
  if (s != CP_OK) return s;
  const bool mixed = prec == CP_MIXED;
  if ((s = check_tensor(ctx, Z, !mixed, mixed, "Z")) != CP_OK) return s;
  if ((s = require_dense(ctx, Z, "timing and tuning calls")) != CP_OK) return s;
  const int N = Z->order;
  if ((s = check_factors(ctx, A, N, mixed, "A")) != CP_OK) return s;
  if (reps < 1 || reps > 10000) return set_err(ctx, CP_ERR_INVALID, "cp_autotune: reps outside [1, 10000]");
  const int R = A->rank;
  const void* z = mixed ? (const void*)Z->z32 : (const void*)Z->z64;
  // candidate options per mode
  std::vector<std::vector<PlanOpts>> cands(N);
  size_t maxpart = 0;
  for (int n = 0; n < N; ++n) {
    const MttkrpPlan p0 = mttkrp_plan(N, Z->dims, n, R, mixed, PlanOpts{kTargetWgs, 0, 2, 4});
    const int kss[] = {0, 1, 2, 4, 8, 16};
    const int tws1[] = {2};
    const int tws23[] = {2, 4};
    const int* tws = p0.kind == 1 ? tws1 : tws23;
    const int ntw = p0.kind == 1 ? 1 : (p0.nt == 1 ? 2 : 1);
    for (int pf = 0; pf < (mixed ? 2 : 1); ++pf) {   // pf: FP32 lane width 4 or 8
      const int vwo = pf ? 8 : 4;
      const int cap = mttkrp_capacity(mttkrp_plan(N, Z->dims, n, R, mixed, PlanOpts{kTargetWgs, 0, 2, vwo}), mixed);
      const int targets[] = {cap - 1, cap / 2 - 1, 2 * cap - 1, (3 * cap) / 4 - 1, cap / 4 - 1};
      for (int t : targets) {
        if (t < 1) continue;
        for (int ks : kss)
          for (int q = 0; q < ntw; ++q)
            for (int ns = 0; ns < 2; ++ns) {
              PlanOpts o{t, ks, tws[q], vwo, ns};
              const MttkrpPlan p = mttkrp_plan(N, Z->dims, n, R, mixed, o);
              if (p.ksplit != ks && ks != 0) continue;   // clamped duplicate
              if (ns && !p0.bl) continue;                 // never staged anyway
              cands[n].push_back(o);
              maxpart = std::max(maxpart, p.partial_doubles);
            }
      }
    }
  }
  // with the dimension tree, the mode-1 launch of a sweep also stores Y: its
  // candidates (the contraction in one piece, factor staged) are timed as well
  size_t ydoubles = 0;
  std::vector<PlanOpts> ycands;
  if (ctx->dimtree && N >= 3) {
    int64_t S = 1, P = 1;
    for (int m = 2; m < N; ++m) S *= Z->dims[m];
    for (int m = 0; m < N; ++m) P *= Z->dims[m];
    const size_t yd = (size_t)S * Z->dims[1] * R;
    if (yd * 8 * 4 <= (size_t)P * (mixed ? 4 : 8)) {
      for (PlanOpts o : cands[1]) {
        o.ksplit = 1;
        o.nostage = 0;
        const MttkrpPlan p = mttkrp_plan(N, Z->dims, 1, R, mixed, o);
        if (p.ksplit != 1) continue;
        bool dup = false;
        for (const PlanOpts& q : ycands)
          dup = dup || (q.target_wgs == o.target_wgs && q.tw == o.tw && q.vw == o.vw);
        if (dup) continue;
        ycands.push_back(o);
        maxpart = std::max(maxpart, p.partial_doubles);
      }
      if (!ycands.empty()) ydoubles = yd;
    }
  }
  Sizer sz;
  sz.take<double>((size_t)N * R * R);
  sz.take<double>((size_t)N * R);
  sz.take<double>(maxpart);
  sz.take<double>(ydoubles);
  if ((s = ensure_ws(ctx, sz.off)) != CP_OK) return s;
  Arena ar(ctx->ws);
  double* grams = ar.take<double>((size_t)N * R * R);
  double* sigma = ar.take<double>((size_t)N * R);
  double* part = ar.take<double>(maxpart);
  double* y = ydoubles ? ar.take<double>(ydoubles) : nullptr;
  HIPCHK(gram_launch(A->a, nullptr, Z->dims, N, R, grams, ctx->stream, sigma));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  std::ostringstream report;
  for (int pass = 0; pass <= N; ++pass) {
    // passes 0..N-1: the plain launch of mode `pass`; pass N: mode 1 storing Y
    const bool ys = pass == N;
    if (ys && !y) break;
    const int n = ys ? 1 : pass;
    const PrepArgs pa = timing_prep(ctx, Z, A, n, grams, sigma);
    double best = 1e30;
    PlanOpts bo{};
    for (const PlanOpts& o : ys ? ycands : cands[n]) {
      const MttkrpPlan p = mttkrp_plan(N, Z->dims, n, R, mixed, o);
      for (int w = 0; w < 2; ++w)
        HIPCHK(mttkrp_launch(p, Z->dims, N, n, R, z, mixed, A->a, (const float* const*)A->a32, part,
                             &pa, ctx->stream, ys ? y : nullptr));
      HIPCHK(hipEventRecord(e0, ctx->stream));
      for (int k = 0; k < reps; ++k)
        HIPCHK(mttkrp_launch(p, Z->dims, N, n, R, z, mixed, A->a, (const float* const*)A->a32, part,
                             &pa, ctx->stream, ys ? y : nullptr));
      HIPCHK(hipEventRecord(e1, ctx->stream));
      HIPCHK(hipEventSynchronize(e1));
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, e0, e1));
      const double us = 1e3 * t / reps;
      if (us < best) {
        best = us;
        bo = o;
      }
    }
    const std::string key = plan_key(N, Z->dims, n, R, mixed) + (ys ? ";y" : "");
    ctx->tuned[key] = bo;
    ctx->plans.erase(key);
    report << key << " " << bo.target_wgs << " " << bo.ksplit << " " << bo.tw << " " << bo.vw << " "
           << bo.nostage
           << " " << best << "\n";
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return CP_OK;
}

const char* cp_plans_export(cp_ctx ctx) {
  if (!ctx) return "";
  std::ostringstream o;
  for (const auto& kv : ctx->tuned)
    o << kv.first << " " << kv.second.target_wgs << " " << kv.second.ksplit << " " << kv.second.tw
      << " " << kv.second.vw << " " << kv.second.nostage << "\n";
  ctx->plans_text = o.str();
  return ctx->plans_text.c_str();
}

cp_status cp_plans_import(cp_ctx ctx, const char* text) {
  if (!ctx) return CP_ERR_INVALID;
  if (!text) return set_err(ctx, CP_ERR_INVALID, "cp_plans_import: NULL text");
  std::istringstream in(text);
  std::string line;
  int count = 0;
  while (std::getline(in, line)) {
    if (line.empty()) continue;
    std::istringstream ls(line);
    std::string key;
    PlanOpts o{};
    if (!(ls >> key >> o.target_wgs >> o.ksplit >> o.tw >> o.vw) || o.target_wgs < 1 ||
        o.ksplit < 0 || (o.tw != 2 && o.tw != 4) || (o.vw != 4 && o.vw != 8))
      return set_err(ctx, CP_ERR_INVALID, "cp_plans_import: bad line '%s'", line.c_str());
    if (!(ls >> o.nostage)) o.nostage = 0;   // optional last field
    if (o.nostage != 0 && o.nostage != 1)
      return set_err(ctx, CP_ERR_INVALID, "cp_plans_import: bad line '%s'", line.c_str());
    ctx->tuned[key] = o;
    ctx->plans.erase(key);
    ++count;
  }
  return CP_OK;
}

cp_status cp_profile_enable(cp_ctx ctx, int32_t on) {
  if (!ctx) return CP_ERR_INVALID;
  if (on) {
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (auto& r : ctx->recs) {
      ctx->pool.push_back(r.a);
      ctx->pool.push_back(r.b);
    }
    ctx->recs.clear();
  }
  ctx->prof = on != 0;
  return CP_OK;
}

cp_status cp_profile_read(cp_ctx ctx, double* ms, int32_t* counts) {
  if (!ctx) return CP_ERR_INVALID;
  if (!ms || !counts) return set_err(ctx, CP_ERR_INVALID, "cp_profile_read: NULL output");
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < CP_PROF_CLASSES; ++k) {
    ms[k] = 0.0;
    counts[k] = 0;
  }
  for (auto& r : ctx->recs) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.cls] += t;
    counts[r.cls] += 1;
    ctx->pool.push_back(r.a);
    ctx->pool.push_back(r.b);
  }
  ctx->recs.clear();
  return CP_OK;
}

cp_status cp_sort(cp_ctx ctx, const int64_t* dims, int32_t order, cp_factors* A) {
  if (!ctx) return CP_ERR_INVALID;
  if (!dims) return set_err(ctx, CP_ERR_INVALID, "cp_sort: dims is NULL");
  if (order < 1 || order > CP_MAX_ORDER) return set_err(ctx, CP_ERR_SHAPE, "cp_sort: bad order");
  cp_status s = check_factors(ctx, A, order, false, "A");
  if (s != CP_OK) return s;
  bool have32 = true;
  for (int m = 0; m < order; ++m) have32 = have32 && A->a32[m];
  HIPCHK(sort_launch(A->a, have32 ? A->a32 : nullptr, dims, order, A->rank, nullptr, ctx->stream));
  return CP_OK;
}

}  // extern "C"

// ===========================================================================
// CP-FAS V-cycle (Algorithm 2).  Host recursion over the levels; every step is
// a kernel enqueued on the context's stream.
namespace {

struct FasLevel {
  int64_t dims[CP_MAX_ORDER];
  const void* z = nullptr;
  const double* phat[CP_MAX_ORDER] = {};
  double* A[CP_MAX_ORDER] = {};
  float* A32[CP_MAX_ORDER] = {};
  double* At[CP_MAX_ORDER] = {};
  double* F[CP_MAX_ORDER] = {};
  double* H[CP_MAX_ORDER] = {};
  double* grams = nullptr;
  SweepPlan sp;
  bool has32 = false;
  bool sparse = false;   // level tensor in the sparse form (level 0 only)
  SpTensor spt{};
  const SpTensor* spp() const { return sparse ? &spt : nullptr; }
};

struct FasRun {
  cp_ctx ctx;
  int N, R, L;
  bool mixed;
  cp_fas_params p;
  std::vector<FasLevel> lv;
  double* partial;
  double* gram_part;
  double* scal_part;
  double* sigma;
  double* y;
};

cp_status fas_relax(FasRun& r, int l, int times) {
  cp_ctx ctx = r.ctx;
  FasLevel& L = r.lv[l];
  cp_status st = CP_OK;
  if (l > 0 && try_small_relax(ctx, L.dims, r.N, r.R, L.z, r.mixed, L.A, L.has32 ? L.A32 : nullptr, L.F,
                               r.p.gs_iters, times, &st))
    return st;
  SweepWS w{L.grams, r.sigma, r.partial, r.gram_part, r.scal_part, L.sp.dimtree ? r.y : nullptr};
  return enqueue_sweeps(ctx, L.dims, r.N, r.R, L.z, r.mixed, L.A, L.has32 ? L.A32 : nullptr,
                        l == 0 ? nullptr : L.F, L.sp, w, CP_SOLVE_GS, r.p.gs_iters,
                        l == 0 ? 1 : 0, times, nullptr, nullptr, L.spp());
}

// H^(n)(A) = A^(n) Gamma^(n) - Z_(n) Phi^(n) for every mode of level l.
cp_status fas_H(FasRun& r, int l, double* const* A, float* const* A32, double* const* Hout) {
  cp_ctx ctx = r.ctx;
  FasLevel& L = r.lv[l];
  TRY(enqueue_gram(ctx, A, A32, L.dims, r.N, r.R, L.grams));
  for (int n = 0; n < r.N; ++n) {
    cp_status s = enqueue_mttkrp(ctx, L.dims, r.N, n, r.R, L.z, r.mixed, (const double* const*)A,
                                 (const float* const*)A32, L.sp.p[n], r.partial, nullptr, L.spp());
    if (s != CP_OK) return s;
    EpiDesc d{};
    d.op = EPI_H;
    d.R = r.R;
    d.N = r.N;
    d.n = n;
    d.nsplit = L.sp.p[n].nsplit;
    d.In = L.dims[n];
    d.partial = r.partial;
    d.A = A[n];
    d.grams = L.grams;
    d.outbuf = Hout[n];
    TRY(enqueue_epi(ctx, d));
  }
  return CP_OK;
}

// Run `body` (which enqueues on ctx->stream) as a HIP graph: recorded on the
// context's private capture stream the first time `key` is seen, replayed on
// the context's stream after that.  A capture that fails leaves graphs off for
// this context and runs `body` directly.
template <typename F>
cp_status run_graph(cp_ctx ctx, const std::string& key, F&& body) {
  auto hit = ctx->gcache.find(key);
  if (hit != ctx->gcache.end()) {
    HIPCHK(hipGraphLaunch(hit->second, ctx->stream));
    return CP_OK;
  }
  if (ctx->gcache.size() >= 32) clear_graphs(ctx);
  if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  hipStream_t user = ctx->stream;
  ctx->stream = ctx->cap_stream;
  hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    ctx->stream = user;
    ctx->graphs = 0;
    return body();
  }
  const cp_status sb = body();
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(ctx->cap_stream, &g);
  ctx->stream = user;
  if (sb != CP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return sb;
  }
  hipGraphExec_t ex = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ctx->graphs = 0;
    return body();
  }
  ctx->gcache[key] = ex;
  HIPCHK(hipGraphLaunch(ex, ctx->stream));
  return CP_OK;
}

cp_status fas_vcycle_rec(FasRun& r, int l) {
  cp_ctx ctx = r.ctx;
  if (l == r.L - 1) return fas_relax(r, l, r.p.nuc);
  cp_status s = fas_relax(r, l, r.p.nu1);
  if (s != CP_OK) return s;
  FasLevel& cur = r.lv[l];
  FasLevel& nx = r.lv[l + 1];
  const int R = r.R;
  // coarse initial guess A~_c (eq. (21))
  for (int n = 0; n < r.N; ++n)
    HIPCHK(restrict_factor_launch(cur.dims[n], nx.dims[n], R, cur.phat[n], cur.A[n], nx.At[n],
                                  ctx->stream));
  // H(A) on this level and H_c(A~_c) on the next
  if ((s = fas_H(r, l, cur.A, cur.has32 ? cur.A32 : nullptr, cur.H)) != CP_OK) return s;
  if ((s = fas_H(r, l + 1, nx.At, nx.has32 ? nx.A32 : nullptr, nx.H)) != CP_OK) return s;
  // coarse right-hand side (eq. (27)); modes that are not coarsened use ic_rule
  for (int n = 0; n < r.N; ++n) {
    const double* F = (l == 0) ? nullptr : cur.F[n];
    if (cur.phat[n])
      HIPCHK(fas_rhs_launch(cur.dims[n], nx.dims[n], R, cur.phat[n], F, cur.H[n], nx.H[n], nx.F[n],
                            ctx->stream));
    else
      HIPCHK(fas_rhs_identity_launch(cur.dims[n] * R, F, cur.H[n], nx.H[n], r.p.ic_rule, nx.F[n],
                                     ctx->stream));
    HIPCHK(copy_launch(nx.At[n], nx.A[n], nx.dims[n] * R, ctx->stream));
  }
  if ((s = fas_vcycle_rec(r, l + 1)) != CP_OK) return s;
  // coarse-grid correction (eq. (28))
  for (int n = 0; n < r.N; ++n)
    HIPCHK(prolong_launch(cur.dims[n], nx.dims[n], R, cur.phat[n], nx.A[n], nx.At[n], cur.A[n],
                          ctx->stream));
  return fas_relax(r, l, r.p.nu2);
}

}  // namespace

extern "C" cp_status cp_fas_vcycle(cp_ctx ctx, const cp_level* levels, int32_t nlevels,
                                   cp_factors* A, const cp_fas_params* params, cp_prec prec) {
  if (!ctx) return CP_ERR_INVALID;
  cp_status s = check_prec(ctx, prec);
  if (s != CP_OK) return s;
  const bool mixed = prec == CP_MIXED;
  if (!levels || nlevels < 1) return set_err(ctx, CP_ERR_INVALID, "cp_fas_vcycle: no levels");
  const int N = levels[0].z.order;
  for (int l = 0; l < nlevels; ++l) {
    char name[32];
    snprintf(name, sizeof(name), "levels[%d].z", l);
    if ((s = check_tensor(ctx, &levels[l].z, !mixed, mixed, name)) != CP_OK) return s;
    if (l > 0 && levels[l].z.nnz != 0)
      return set_err(ctx, CP_ERR_UNSUPPORTED, "level %d: only level 0 may be in the sparse form", l);
    if (levels[l].z.order != N) return set_err(ctx, CP_ERR_SHAPE, "level %d has order %d != %d", l, levels[l].z.order, N);
    if (l + 1 < nlevels) {
      for (int n = 0; n < N; ++n) {
        const int64_t want = levels[l].phat[n] ? (levels[l].z.dims[n] + 1) / 2 : levels[l].z.dims[n];
        if (levels[l + 1].z.dims[n] != want)
          return set_err(ctx, CP_ERR_SHAPE, "level %d mode %d: dims %lld, expected %lld", l + 1, n,
                         (long long)levels[l + 1].z.dims[n], (long long)want);
      }
    }
  }
  if ((s = check_factors(ctx, A, N, mixed, "A")) != CP_OK) return s;
  cp_fas_params p{1, 1, 50, 10, 0};
  if (params) p = *params;
  if (p.nu1 < 0 || p.nu2 < 0 || p.nuc < 0 || p.gs_iters < 1 || p.gs_iters > 1000 ||
      (p.ic_rule != 0 && p.ic_rule != 1))
    return set_err(ctx, CP_ERR_INVALID, "cp_fas_vcycle: bad parameters");
  const int R = A->rank;
  FasRun r{ctx, N, R, nlevels, mixed, p, std::vector<FasLevel>(nlevels), nullptr, nullptr, nullptr,
           nullptr, nullptr};
  bool have32 = true;
  for (int m = 0; m < N; ++m) have32 = have32 && A->a32[m];
  size_t maxpart = 0, maxy = 0;
  int64_t maxI = 0;
  for (int l = 0; l < nlevels; ++l) {
    FasLevel& L = r.lv[l];
    for (int n = 0; n < N; ++n) {
      L.dims[n] = levels[l].z.dims[n];
      L.phat[n] = (l + 1 < nlevels) ? levels[l].phat[n] : nullptr;
    }
    L.z = mixed ? (const void*)levels[l].z.z32 : (const void*)levels[l].z.z64;
    L.sparse = is_sparse(&levels[l].z);
    if (L.sparse) L.spt = sp_view(&levels[l].z);
    L.sp = sweep_plan(ctx, L.dims, N, R, mixed, L.spp());
    maxpart = std::max(maxpart, L.sp.partial);
    maxy = std::max(maxy, L.sp.ydoubles);
    maxI = std::max(maxI, max_dim(L.dims, N));
  }
  auto carve = [&](auto& c, bool real) {
    for (int l = 0; l < nlevels; ++l) {
      FasLevel& L = r.lv[l];
      for (int n = 0; n < N; ++n) {
        const size_t cnt = (size_t)L.dims[n] * R;
        if (l >= 1) {
          double* a = c.template take<double>(cnt);
          double* at = c.template take<double>(cnt);
          double* f = c.template take<double>(cnt);
          float* a32 = (mixed || have32) ? c.template take<float>(cnt) : nullptr;
          if (real) { L.A[n] = a; L.At[n] = at; L.F[n] = f; L.A32[n] = a32; }
        }
        double* h = c.template take<double>(cnt);
        if (real) L.H[n] = h;
      }
      double* g = c.template take<double>((size_t)N * R * R);
      if (real) L.grams = g;
    }
    double* part = c.template take<double>(maxpart);
    const int64_t nwg = epi_blocks(maxI);
    double* gp = c.template take<double>((size_t)nwg * R * R);
    double* sp = c.template take<double>((size_t)std::max<int64_t>(nwg, 2048));
    double* sg = c.template take<double>((size_t)N * R);
    double* yb = maxy ? c.template take<double>(maxy) : nullptr;
    if (real) { r.partial = part; r.gram_part = gp; r.scal_part = sp; r.sigma = sg; r.y = yb; }
  };
  Sizer sz;
  carve(sz, false);
  if ((s = ensure_ws(ctx, sz.off)) != CP_OK) return s;
  Arena ar(ctx->ws);
  carve(ar, true);
  for (int n = 0; n < N; ++n) {
    r.lv[0].A[n] = A->a[n];
    r.lv[0].A32[n] = A->a32[n];
  }
  for (int l = 0; l < nlevels; ++l) r.lv[l].has32 = (l == 0) ? have32 : (mixed || have32);
  auto body = [&]() -> cp_status {
    cp_status t = fas_vcycle_rec(r, 0);
    if (t != CP_OK) return t;
    if (r.lv[0].has32)   // shadows of the finest factors follow the last correction
      return enqueue_gram(ctx, A->a, A->a32, r.lv[0].dims, N, R, r.lv[0].grams);
    return CP_OK;
  };
  if (!ctx->graphs || ctx->prof) return body();
  // the launch sequence depends only on these arguments and the workspace
  std::ostringstream key;
  key << "fas;" << nlevels << ";" << N << ";" << R << ";" << (int)mixed << ";" << p.nu1 << "," << p.nu2 << ","
      << p.nuc << "," << p.gs_iters << "," << p.ic_rule << ";" << (const void*)ctx->ws << ";" << ctx->ws_cap << ";"
      << ctx->dimtree;
  for (int l = 0; l < nlevels; ++l) {
    key << "|" << r.lv[l].z;
    if (r.lv[l].sparse) {
      const SpTensor& t = r.lv[l].spt;
      key << ",sp" << t.nnz << "," << (const void*)t.idx << "," << (const void*)t.vals;
      for (int n = 0; n < N; ++n) key << "," << (const void*)t.rowptr[n] << "," << (const void*)t.perm[n];
    }
    for (int n = 0; n < N; ++n) key << "," << r.lv[l].dims[n] << "," << (const void*)r.lv[l].phat[n];
  }
  for (int n = 0; n < N; ++n) key << "|" << (const void*)A->a[n] << "," << (const void*)A->a32[n];
  return run_graph(ctx, key.str(), body);
}

// ===========================================================================
// Batched solves
// ===========================================================================
namespace {

// Tensor bytes one streaming workgroup of a batched MTTKRP aims to cover.
constexpr int64_t kBatchBytesPerWg = 192 * 1024;   // default of cp_batch_params::wg_kib
// Mixed form: below this many active problems the FP32-phase ones move to FP64.
constexpr int kBatchMergeBelow = 64;

struct BatchPhase {           // device arrays of one phase (FP32 or FP64 contractions)
  MttkrpDesc* md = nullptr;   // [(N + 1) * nprob]: set 0 = first sweep of a chunk, mode 0;
                              // set 1 + n = mode n of the other sweeps
  EpiDesc* ed = nullptr;      // [N * nprob]
  PrepArgs* fin = nullptr;    // [nprob]
  std::vector<std::vector<int2*>> mtiles;   // [set][nt-1]
  std::vector<std::vector<int>> mcount;
  std::vector<std::vector<size_t>> msmem;
  std::vector<int2*> etiles;                // [n]
  std::vector<int> ecount;
};

}  // namespace

extern "C" cp_status cp_als_batched(cp_ctx ctx, const cp_batch_problem* probs, int32_t nprob,
                                    const cp_batch_params* prm, double* fits, int32_t* sweeps) {
  if (!ctx) return CP_ERR_INVALID;
  if (!probs || nprob < 1) return set_err(ctx, CP_ERR_INVALID, "cp_als_batched: no problems");
  if (!prm) return set_err(ctx, CP_ERR_INVALID, "cp_als_batched: params NULL");
  cp_status s = check_prec(ctx, prm->prec);
  if (s != CP_OK) return s;
  const int G = prm->restarts;
  if (G < 1 || G > CP_MAX_RESTARTS || G > kMaxGroups)
    return set_err(ctx, CP_ERR_INVALID, "cp_als_batched: restarts %d outside [1, %d]", G, CP_MAX_RESTARTS);
  if (prm->window32 < 2 || prm->max_sweeps < 1 || prm->chunk < 1 || !(prm->tol32 >= 0.0) ||
      !(prm->tol64 >= 0.0))
    return set_err(ctx, CP_ERR_INVALID, "cp_als_batched: window32 >= 2, max_sweeps >= 1, chunk >= 1 "
                                        "and non-negative tolerances required");
  if (prm->wg_kib != 0 && (prm->wg_kib < 16 || prm->wg_kib > 4096))
    return set_err(ctx, CP_ERR_INVALID, "cp_als_batched: wg_kib %d outside [16, 4096] (0 = default)", prm->wg_kib);
  const int64_t wg_bytes = prm->wg_kib ? (int64_t)prm->wg_kib * 1024 : kBatchBytesPerWg;
  const bool mixed = prm->prec == CP_MIXED;
  int N = 0;
  for (int b = 0; b < nprob; ++b) {
    const cp_batch_problem& pb = probs[b];
    if ((s = check_tensor(ctx, &pb.z, true, mixed, "problem tensor")) != CP_OK) return s;
    if ((s = require_dense(ctx, &pb.z, "cp_als_batched")) != CP_OK) return s;
    if (b == 0) N = pb.z.order;
    if (pb.z.order != N)
      return set_err(ctx, CP_ERR_SHAPE, "cp_als_batched: problem %d has order %d, problem 0 has %d", b,
                     pb.z.order, N);
    if (!pb.z.norm2) return set_err(ctx, CP_ERR_INVALID, "cp_als_batched: problem %d: norm2 NULL", b);
    if ((s = check_factors(ctx, &pb.a, N, mixed, "problem factors")) != CP_OK) return s;
    if (pb.a.rank % G != 0)
      return set_err(ctx, CP_ERR_SHAPE, "cp_als_batched: problem %d: rank %d is not a multiple of %d restarts",
                     b, pb.a.rank, G);
  }
  const int nphase = mixed ? 2 : 1;
  const int nsets = N + 1;

  // ---- launch plans, per problem, mode and phase -------------------------
  // plans[ph][b * N + n]
  std::vector<std::vector<MttkrpPlan>> plans(nphase, std::vector<MttkrpPlan>((size_t)nprob * N));
  std::vector<size_t> maxpart(nprob, 0);
  for (int ph = 0; ph < nphase; ++ph) {
    const bool fp32 = mixed && ph == 0;
    for (int b = 0; b < nprob; ++b) {
      const cp_batch_problem& pb = probs[b];
      int64_t P = 1;
      for (int m = 0; m < N; ++m) P *= pb.z.dims[m];
      const int64_t bytes = P * (fp32 ? 4 : 8);
      const int target = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (bytes + wg_bytes - 1) / wg_bytes));
      for (int n = 0; n < N; ++n) {
        MttkrpPlan p = mttkrp_plan(N, pb.z.dims, n, pb.a.rank, fp32, PlanOpts{target, 0, 2, 4});
        if (!p.bl)
          return set_err(ctx, CP_ERR_UNSUPPORTED,
                         "cp_als_batched: problem %d: contracted mode too large to stage in LDS", b);
        plans[ph][(size_t)b * N + n] = p;
        maxpart[b] = std::max(maxpart[b], p.partial_doubles);
      }
    }
  }

  // ---- tiles (host) --------------------------------------------------------
  struct HostPhase {
    std::vector<std::vector<std::vector<int2>>> mt;   // [set][nt-1]
    std::vector<std::vector<size_t>> msmem;
    std::vector<std::vector<int2>> et;                // [n]
  };
  std::vector<HostPhase> hp(nphase);
  for (int ph = 0; ph < nphase; ++ph) {
    HostPhase& h = hp[ph];
    h.mt.assign(nsets, std::vector<std::vector<int2>>(2));
    h.msmem.assign(nsets, std::vector<size_t>(2, 0));
    h.et.assign(N, {});
    for (int set = 0; set < nsets; ++set) {
      const int n = set == 0 ? 0 : set - 1;
      for (int b = 0; b < nprob; ++b) {
        const MttkrpPlan& p = plans[ph][(size_t)b * N + n];
        const int nt = p.nt;
        const int64_t grid = (int64_t)p.ngroups * p.nsplit + 1;
        for (int64_t t = 0; t < grid; ++t) h.mt[set][nt - 1].push_back(int2{set * nprob + b, (int)t});
        h.msmem[set][nt - 1] =
            std::max(h.msmem[set][nt - 1], mttkrp_smem_bytes(p, N, probs[b].a.rank, true));
      }
    }
    for (int n = 0; n < N; ++n)
      for (int b = 0; b < nprob; ++b) {
        const int64_t nb = epi_blocks(probs[b].z.dims[n]);
        for (int64_t t = 0; t < nb; ++t) h.et[n].push_back(int2{n * nprob + b, (int)t});
      }
  }

  // ---- workspace -----------------------------------------------------------
  std::vector<double*> grams(nprob), sigma(nprob), part(nprob), scal(nprob), pout(nprob);
  std::vector<int32_t*> ckind(nprob);
  BatchState* states = nullptr;
  BatchRule* rules = nullptr;
  std::vector<BatchPhase> dp(nphase);
  GramJob* jobs = nullptr;
  int32_t* plist = nullptr;
  int smem_fin = 0;
  auto carve = [&](auto& c, bool real) {
    for (int b = 0; b < nprob; ++b) {
      const int R = probs[b].a.rank;
      double* g = c.template take<double>((size_t)N * R * R);
      double* sg = c.template take<double>((size_t)N * R);
      double* pt = c.template take<double>(maxpart[b]);
      double* sc = c.template take<double>((size_t)epi_blocks(probs[b].z.dims[N - 1]) * G);
      double* po = c.template take<double>((size_t)R * R + 2 * R);
      int32_t* ck = c.template take<int32_t>(1);
      if (real) { grams[b] = g; sigma[b] = sg; part[b] = pt; scal[b] = sc; pout[b] = po; ckind[b] = ck; }
    }
    BatchState* stp = c.template take<BatchState>((size_t)nprob);
    BatchRule* ru = c.template take<BatchRule>(2);
    GramJob* jb = c.template take<GramJob>((size_t)nprob * N);
    int32_t* pl = c.template take<int32_t>((size_t)nprob * 3);
    if (real) { states = stp; rules = ru; jobs = jb; plist = pl; }
    for (int ph = 0; ph < nphase; ++ph) {
      MttkrpDesc* md = c.template take<MttkrpDesc>((size_t)nsets * nprob);
      EpiDesc* ed = c.template take<EpiDesc>((size_t)N * nprob);
      PrepArgs* fin = c.template take<PrepArgs>((size_t)nprob);
      if (real) { dp[ph].md = md; dp[ph].ed = ed; dp[ph].fin = fin; }
      if (real) {
        dp[ph].mtiles.assign(nsets, std::vector<int2*>(2, nullptr));
        dp[ph].mcount.assign(nsets, std::vector<int>(2, 0));
        dp[ph].msmem = hp[ph].msmem;
        dp[ph].etiles.assign(N, nullptr);
        dp[ph].ecount.assign(N, 0);
      }
      for (int set = 0; set < nsets; ++set)
        for (int q = 0; q < 2; ++q) {
          int2* t = c.template take<int2>(hp[ph].mt[set][q].size());
          if (real) { dp[ph].mtiles[set][q] = t; dp[ph].mcount[set][q] = (int)hp[ph].mt[set][q].size(); }
        }
      for (int n = 0; n < N; ++n) {
        int2* t = c.template take<int2>(hp[ph].et[n].size());
        if (real) { dp[ph].etiles[n] = t; dp[ph].ecount[n] = (int)hp[ph].et[n].size(); }
      }
    }
  };
  Sizer sz;
  carve(sz, false);
  if ((s = ensure_ws(ctx, sz.off)) != CP_OK) return s;
  Arena ar(ctx->ws);
  carve(ar, true);
  for (int b = 0; b < nprob; ++b) smem_fin = std::max(smem_fin, prep_smem_doubles(N, probs[b].a.rank));

  // ---- descriptors (host), then one upload --------------------------------
  BatchRule hr[2];
  for (int ph = 0; ph < 2; ++ph) {
    hr[ph] = BatchRule{};
    hr[ph].phase = ph;
    hr[ph].window = prm->window32;
    hr[ph].tol32 = prm->tol32;
    hr[ph].tol64 = prm->tol64;
    hr[ph].max_sweeps = prm->max_sweeps;
  }
  // rule index of launch phase ph: the mixed form runs FP32 (0) and FP64 (1)
  // launches, the FP64 form only FP64 (1)
  auto run_phase = [&](int ph) { return (mixed && ph == 0) ? 0 : 1; };
  auto phase_rule = [&](int ph) { return rules + run_phase(ph); };
  std::vector<GramJob> hjobs((size_t)nprob * N);
  for (int b = 0; b < nprob; ++b)
    for (int n = 0; n < N; ++n) {
      const int R = probs[b].a.rank;
      GramJob j{};
      j.A = probs[b].a.a[n];
      j.A32 = mixed ? probs[b].a.a32[n] : nullptr;
      j.I = probs[b].z.dims[n];
      j.R = R;
      j.gram = grams[b] + (size_t)n * R * R;
      j.sigma = sigma[b] + (size_t)n * R;
      j.st = states + b;
      hjobs[(size_t)b * N + n] = j;
    }
  std::vector<std::vector<MttkrpDesc>> hmd(nphase);
  std::vector<std::vector<EpiDesc>> hed(nphase);
  std::vector<std::vector<PrepArgs>> hfin(nphase);
  for (int ph = 0; ph < nphase; ++ph) {
    const bool fp32 = mixed && ph == 0;
    hmd[ph].resize((size_t)nsets * nprob);
    hed[ph].resize((size_t)N * nprob);
    hfin[ph].resize(nprob);
    for (int b = 0; b < nprob; ++b) {
      const cp_batch_problem& pb = probs[b];
      const int R = pb.a.rank;
      auto base = [&](int n) {
        PrepArgs pa{};
        pa.N = N;
        pa.n = n;
        pa.R = R;
        pa.grams = grams[b];
        pa.sigma = sigma[b];
        pa.out = pout[b];
        pa.kind = ckind[b];
        pa.flags = ctx->flags;
        pa.solver = CP_SOLVE_CHOL;
        pa.normalize = 1;
        pa.norm2 = pb.z.norm2;
        pa.inner_part = scal[b];
        pa.inner_count = (int32_t)epi_blocks(pb.z.dims[N - 1]);
        pa.groups = G;
        pa.st = states + b;
        pa.rule = phase_rule(ph);
        pa.run_phase = run_phase(ph);
        return pa;
      };
      const void* z = fp32 ? (const void*)pb.z.z32 : (const void*)pb.z.z64;
      for (int set = 0; set < nsets; ++set) {
        const int n = set == 0 ? 0 : set - 1;
        PrepArgs pa = base(n);
        if (set == 0) {
          pa.p = -1;
        } else {
          pa.p = (n + N - 1) % N;
          pa.Ap = pb.a.a[pa.p];
          pa.Ip = pb.z.dims[pa.p];
          pa.boundary = n == 0 ? 1 : 0;
        }
        hmd[ph][(size_t)set * nprob + b] =
            mttkrp_desc(plans[ph][(size_t)b * N + n], pb.z.dims, N, n, R, z, fp32, pb.a.a,
                        (const float* const*)pb.a.a32, part[b], &pa);
      }
      for (int n = 0; n < N; ++n) {
        EpiDesc d{};
        d.op = EPI_UPDATE;
        d.solver = CP_SOLVE_CHOL;
        d.gs_iters = 10;
        d.R = R;
        d.N = N;
        d.n = n;
        d.nsplit = plans[ph][(size_t)b * N + n].nsplit;
        d.In = pb.z.dims[n];
        d.partial = part[b];
        d.A = pb.a.a[n];
        d.A32 = mixed ? pb.a.a32[n] : nullptr;
        d.grams = grams[b];
        d.prep_out = pout[b];
        d.kind = ckind[b];
        d.scal_part = scal[b];
        d.flags = ctx->flags;
        d.want_obj = n == N - 1 ? 1 : 0;
        d.groups = G;
        d.st = states + b;
        d.run_phase = run_phase(ph);
        hed[ph][(size_t)n * nprob + b] = d;
      }
      PrepArgs fa = base(0);
      fa.p = N - 1;
      fa.Ap = pb.a.a[N - 1];
      fa.Ip = pb.z.dims[N - 1];
      fa.boundary = 1;
      for (int m = 0; m < N; ++m) {
        fa.A[m] = pb.a.a[m];
        fa.A32[m] = mixed ? pb.a.a32[m] : nullptr;
        fa.dims[m] = pb.z.dims[m];
      }
      fa.lds = prep_smem_doubles(N, R);
      hfin[ph][b] = fa;
    }
  }
  std::vector<BatchState> hst(nprob);
  auto init_states = [&](int phase, bool first) {
    for (int b = 0; b < nprob; ++b) {
      BatchState& x = hst[b];
      if (first) x = BatchState{};
      x.phase = mixed ? 0 : 1;
      x.active = 1;
      x.sweep = 0;
      for (int g = 0; g < kMaxGroups; ++g) {
        x.frozen[g] = g < G ? 0 : 1;
        x.fit_prev[g] = std::numeric_limits<double>::quiet_NaN();
        if (first) x.fit[g] = x.fit_win[g] = std::numeric_limits<double>::quiet_NaN();
      }
    }
    (void)phase;
  };
  init_states(0, true);
  hipStream_t st = ctx->stream;
  HIPCHK(hipMemcpyAsync(rules, hr, sizeof(hr), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(jobs, hjobs.data(), hjobs.size() * sizeof(GramJob), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(states, hst.data(), hst.size() * sizeof(BatchState), hipMemcpyHostToDevice, st));
  for (int ph = 0; ph < nphase; ++ph) {
    HIPCHK(hipMemcpyAsync(dp[ph].md, hmd[ph].data(), hmd[ph].size() * sizeof(MttkrpDesc),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dp[ph].ed, hed[ph].data(), hed[ph].size() * sizeof(EpiDesc),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dp[ph].fin, hfin[ph].data(), hfin[ph].size() * sizeof(PrepArgs),
                          hipMemcpyHostToDevice, st));
    for (int set = 0; set < nsets; ++set)
      for (int q = 0; q < 2; ++q)
        if (!hp[ph].mt[set][q].empty())
          HIPCHK(hipMemcpyAsync(dp[ph].mtiles[set][q], hp[ph].mt[set][q].data(),
                                hp[ph].mt[set][q].size() * sizeof(int2), hipMemcpyHostToDevice, st));
    for (int n = 0; n < N; ++n)
      if (!hp[ph].et[n].empty())
        HIPCHK(hipMemcpyAsync(dp[ph].etiles[n], hp[ph].et[n].data(), hp[ph].et[n].size() * sizeof(int2),
                              hipMemcpyHostToDevice, st));
  }
  HIPCHK(hipStreamSynchronize(st));   // host arrays may go once the uploads are done

  // ---- sweeps ------------------------------------------------------------------
  // Each problem moves from the FP32 to the FP64 phase on the device as soon as
  // all its restarts have left the FP32 phase (batch_rules), so the two phases
  // of different problems run side by side: every chunk launches the FP32
  // tiles of the problems in phase 0 and the FP64 tiles of those in phase 1.
  // Launch lists cover the problems active at the start of a chunk; a problem
  // that stops (or changes phase) inside a chunk leaves its tiles early.  Few
  // active problems: longer chunks between host checks (the rules themselves
  // are applied on the device after every sweep).
  const int kinds[3] = {1, 2, 3};
  int32_t* plist_ph[2] = {plist + nprob, plist + 2 * (size_t)nprob};
  std::vector<std::vector<int32_t>> act(nphase);
  std::vector<int32_t> all;
  for (int b = 0; b < nprob; ++b) act[0].push_back(b);
  std::vector<std::vector<std::vector<int2>>> cmt(nsets, std::vector<std::vector<int2>>(2));
  std::vector<std::vector<int2>> cet(N);
  // a problem sweeps at most max_sweeps + 1 times and idles for at most one
  // chunk at its phase change
  const int64_t max_rounds = 2 * (int64_t)prm->max_sweeps + 16 * (int64_t)prm->chunk + 16;
  std::string last_key;
  for (int64_t rounds = 0; rounds < max_rounds;) {
    int na = 0;
    for (int ph = 0; ph < nphase; ++ph) na += (int)act[ph].size();
    if (na == 0) break;
    if (mixed && !act[0].empty() && !act[1].empty() && na <= kBatchMergeBelow) {
      // few problems left: sweeps cost launches, not bytes, so the problems
      // still in the FP32 phase go on in FP64 and one set of launches remains
      for (int bb : act[0]) {
        BatchState& x = hst[bb];
        x.phase = 1;
        x.sweep = 0;
        x.active = 1;
        for (int g = 0; g < kMaxGroups; ++g) {
          x.frozen[g] = g < G ? 0 : 1;
          x.fit_prev[g] = std::numeric_limits<double>::quiet_NaN();
        }
        HIPCHK(hipMemcpyAsync(states + bb, &x, sizeof(BatchState), hipMemcpyHostToDevice, st));
        act[1].push_back(bb);
      }
      act[0].clear();
      std::sort(act[1].begin(), act[1].end());
    }
    int K = na <= 8 ? prm->chunk * 8 : (na <= 64 ? prm->chunk * 2 : prm->chunk);
    K = (int)std::min<int64_t>(K, max_rounds - rounds);
    all.clear();
    for (int ph = 0; ph < nphase; ++ph) {
      BatchPhase& d = dp[ph];
      all.insert(all.end(), act[ph].begin(), act[ph].end());
      const bool full = (int)act[ph].size() == nprob;
      std::vector<char> on(nprob, 0);
      for (int bb : act[ph]) on[bb] = 1;
      for (int set = 0; set < nsets; ++set)
        for (int q = 0; q < 2; ++q) {
          const std::vector<int2>* src = &hp[ph].mt[set][q];
          if (!full) {
            cmt[set][q].clear();
            for (const int2& t : hp[ph].mt[set][q])
              if (on[t.x % nprob]) cmt[set][q].push_back(t);
            src = &cmt[set][q];
          }
          d.mcount[set][q] = (int)src->size();
          if (!src->empty())
            HIPCHK(hipMemcpyAsync(d.mtiles[set][q], src->data(), src->size() * sizeof(int2),
                                  hipMemcpyHostToDevice, st));
        }
      for (int n = 0; n < N; ++n) {
        const std::vector<int2>* src = &hp[ph].et[n];
        if (!full) {
          cet[n].clear();
          for (const int2& t : hp[ph].et[n])
            if (on[t.x % nprob]) cet[n].push_back(t);
          src = &cet[n];
        }
        d.ecount[n] = (int)src->size();
        if (!src->empty())
          HIPCHK(hipMemcpyAsync(d.etiles[n], src->data(), src->size() * sizeof(int2), hipMemcpyHostToDevice, st));
      }
      if (!act[ph].empty())
        HIPCHK(hipMemcpyAsync(plist_ph[ph], act[ph].data(), act[ph].size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipMemcpyAsync(plist, all.data(), all.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    // the chunk's launches (on ctx->stream, which a graph capture redirects)
    auto body = [&]() -> cp_status {
      hipStream_t s = ctx->stream;
      {
        ProfScope ps(ctx, CP_PROF_GRAM);
        HIPCHK(gram_batched_launch(jobs, plist, na, N, s));
      }
      for (int k = 0; k < K; ++k)
        for (int n = 0; n < N; ++n) {
          const int set = (k == 0 && n == 0) ? 0 : n + 1;
          for (int ph = 0; ph < nphase; ++ph) {
            if (act[ph].empty()) continue;
            BatchPhase& d = dp[ph];
            const bool fp32 = mixed && ph == 0;
            {
              ProfScope ps(ctx, (fp32 ? CP_PROF_MTTKRP_MODE0_F32 : CP_PROF_MTTKRP_MODE0_F64) + kinds[std::min(n, 2)] - 1);
              for (int q = 0; q < 2; ++q)
                HIPCHK(mttkrp_batched_launch(kinds[std::min(n, 2)], fp32, q + 1, d.md, d.mtiles[set][q],
                                             d.mcount[set][q], d.msmem[set][q], s));
            }
            ProfScope ps(ctx, CP_PROF_UPDATE);
            HIPCHK(epi_batched_launch(d.ed, d.etiles[n], d.ecount[n], s));
          }
        }
      for (int ph = 0; ph < nphase; ++ph) {
        if (act[ph].empty()) continue;
        ProfScope ps(ctx, CP_PROF_NORMALIZE);
        HIPCHK(finalize_batched_launch(dp[ph].fin, plist_ph[ph], (int)act[ph].size(), smem_fin, s));
      }
      return CP_OK;
    };
    // A chunk whose launch sequence repeats the previous one (same active
    // problems, tile counts and length: the long tail of a batch) is recorded
    // into a HIP graph once and replayed; the launch arguments are device
    // arrays at fixed workspace addresses that the uploads above refill.
    std::ostringstream key;
    key << "batch;" << (const void*)ctx->ws << ";" << ctx->ws_cap << ";" << nprob << ";" << K << ";" << na;
    for (int ph = 0; ph < nphase; ++ph) {
      key << "|" << act[ph].size();
      for (int set = 0; set < nsets; ++set)
        for (int q = 0; q < 2; ++q) key << "," << dp[ph].mcount[set][q] << ":" << dp[ph].msmem[set][q];
      for (int n = 0; n < N; ++n) key << "," << dp[ph].ecount[n];
    }
    const std::string ks = key.str();
    if (ctx->graphs && !ctx->prof && ks == last_key) {
      TRY(run_graph(ctx, ks, body));
    } else {
      TRY(body());
    }
    last_key = ks;
    rounds += K;
    HIPCHK(hipMemcpyAsync(hst.data(), states, hst.size() * sizeof(BatchState), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));   // also retires the host tile lists uploaded above
    for (int ph = 0; ph < nphase; ++ph) act[ph].clear();
    for (int bb = 0; bb < nprob; ++bb)
      if (hst[bb].active) act[mixed ? hst[bb].phase : 0].push_back(bb);
  }

  // ---- outputs -------------------------------------------------------------------
  HIPCHK(hipMemcpy(hst.data(), states, hst.size() * sizeof(BatchState), hipMemcpyDeviceToHost));
  if (fits) {
    std::vector<double> hf((size_t)nprob * G);
    for (int b = 0; b < nprob; ++b)
      for (int g = 0; g < G; ++g) hf[(size_t)b * G + g] = hst[b].fit[g];
    HIPCHK(hipMemcpyAsync(fits, hf.data(), hf.size() * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  if (sweeps) {
    std::vector<int32_t> hs((size_t)nprob * G * 2);
    for (int b = 0; b < nprob; ++b)
      for (int g = 0; g < G; ++g)
        for (int q = 0; q < 2; ++q) hs[((size_t)b * G + g) * 2 + q] = hst[b].sweeps[q][g];
    HIPCHK(hipMemcpyAsync(sweeps, hs.data(), hs.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return CP_OK;
}

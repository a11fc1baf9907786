// Internal declarations shared by the HIP translation units of libcpamg.
// Not part of the public ABI (see include/cpamg.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/cpamg.h"

namespace cpamg {

constexpr int kMaxOrder = CP_MAX_ORDER;
constexpr int kMaxRank = CP_MAX_RANK;
constexpr int kThreads = 256;   // threads per workgroup for every kernel (4 waves)

// Value of v in lane `lane` (uniform across the wave), via scalar reads of
// the two halves: no LDS crossbar round trip.
__device__ __forceinline__ double wave_bcast(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Row of the 16x16 MFMA result held in element v of a lane in lane group g = l/16
// (column = l % 16).  v_mfma_f64_16x16x4f64 interleaves rows (g + 4v);
// v_mfma_f32_16x16x4f32 gives each lane group four consecutive rows (4g + v).
template <typename T> __device__ __forceinline__ constexpr int mfma_row(int g, int v);
template <> __device__ __forceinline__ constexpr int mfma_row<double>(int g, int v) { return g + 4 * v; }
template <> __device__ __forceinline__ constexpr int mfma_row<float>(int g, int v) { return 4 * g + v; }

// ---------------------------------------------------------------------------
// MTTKRP launch descriptor (passed by value to the kernels)
// ---------------------------------------------------------------------------
// The tensor is viewed as (I0, I1, S): mode 0 (fastest), mode 1, and the
// "stripe" index s over modes 2..N-1 (mode 2 fastest).  Three kernel kinds:
//   kind 1 (n == 0): GEMM rows = i0, contraction over i1, Hadamard weight per stripe
//   kind 2 (n == 1): GEMM rows = i1, contraction over i0, Hadamard weight per stripe
//   kind 3 (n >= 2): GEMM rows = i1, contraction over i0, Hadamard-reduce of the
//                    rows with A^(1) and the stripe weight into output row s_n
// Batched solves: per-problem device state of the stopping rules.  A problem
// carries `groups` independent restarts of rank R/groups side by side (their
// factor blocks are the column groups of one rank-R factor set); Gamma is kept
// block-diagonal over the groups, so the restarts never couple.
constexpr int kMaxGroups = 8;

struct BatchRule {
  int32_t phase;        // 0: FP32 phase (window rule), 1: FP64 phase (per-sweep rule)
  int32_t window;       // FP32 phase: sweeps per window
  double tol32;         // FP32 phase: (fit_end - fit_start) / (window - 1) <= tol32 * fit_end
  double tol64;         // FP64 phase: |fit_k - fit_{k-1}| <= tol64 * fit_k
  int32_t max_sweeps;   // cap on the sweeps of one restart over both phases
};

struct BatchState {
  int32_t phase;                  // rule the problem is under: 0 FP32 window rule, 1 FP64 rule
  int32_t active;                 // some group still iterates in the current phase
  int32_t sweep;                  // sweeps completed in the current phase
  int32_t frozen[kMaxGroups];     // group stopped in the current phase
  int32_t sweeps[2][kMaxGroups];  // sweeps per phase and group
  double fit[kMaxGroups];         // fit after the group's last sweep (fused objective)
  double fit_prev[kMaxGroups];    // fit after the previous sweep (NaN: none yet)
  double fit_win[kMaxGroups];     // FP32 phase: fit at the first sweep of the window
};

// LDS of the bookkeeping step (sweep.hpp), in doubles: five R x R work arrays,
// the N x R column scales and, when the launch provides the room
// (PrepArgs::lds), the N stored Grams.
__host__ __device__ constexpr int prep_min_doubles(int N, int R) { return 5 * R * R + N * R; }
__host__ __device__ constexpr bool prep_stage_grams(int N, int R, int lds) {
  return 5 * R * R + N * R + N * R * R <= lds;
}
__host__ __device__ constexpr int prep_smem_doubles(int N, int R) {
  return 5 * R * R + N * R + (N * R * R <= 4096 ? N * R * R : 0);
}

// Per-mode bookkeeping done by the extra first workgroup of an MTTKRP launch
// (or by the finalize kernel at the end of a call); see sweep.hpp.
struct PrepArgs {
  int32_t N, n, R;
  double* grams;            // [N][R][R] Grams of the stored factors
  double* sigma;            // [N][R] pending column scales: normalized = sigma (.) stored
  double* out;              // [R*R + 2R]: factor / pseudoinverse / Gamma, column scale, sigma^(n)
  int32_t* kind;            // 0 Cholesky factor, 1 pseudoinverse, 2 Gamma (Gauss-Seidel)
  uint32_t* flags;
  int32_t solver;
  int32_t p;                // mode whose Gram is recomputed from its factor (-1: none)
  const double* Ap;
  int64_t Ip;
  int32_t boundary;         // a sweep has just ended: fused objective + normalization scales
  int32_t normalize;
  double* f_slot;           // where that sweep's f goes (NULL: not requested)
  const double* norm2;
  const double* inner_part; // per-block <A^(N), M^(N)> of the last update
  int32_t inner_count;
  double* A[kMaxOrder];     // finalize: factors to scale
  float* A32[kMaxOrder];
  int64_t dims[kMaxOrder];
  int32_t groups;           // column groups (independent restarts); 0 or 1: one group
  BatchState* st;           // batched solves: stopping state (NULL otherwise)
  const BatchRule* rule;
  int32_t run_phase;        // batched solves: the phase (rule index) this launch runs
  int32_t lds;              // doubles of LDS the launch provides (set by the launchers)
};

struct MttkrpDesc {
  const void* z;                  // tensor (T*)
  const void* ak;                 // factor of the contracted mode, in T (B operand)
  const double* a64[kMaxOrder];   // FP64 factors (Hadamard stage)
  double* out;                    // partials [nsplit][I_n][R] (or M when nsplit == 1)
  int64_t I0, I1, S;              // view extents
  int64_t In;                     // extent of the output mode
  int32_t N, n, R;
  int32_t kind;
  // stripe decoding: the stripe index is s = sum_j s_j * sst[j] over stripe modes
  int32_t ns;                     // number of stripe modes (N - 2, >= 0)
  int64_t sext[kMaxOrder];        // extents of stripe modes (modes 2..N-1)
  int64_t sst[kMaxOrder];         // strides in the stripe index
  // work split
  int32_t ngroups;                // kind 1: row panels of 64; kind 2: row groups; kind 3: outputs I_n
  int32_t nsplit;                 // workgroups per group
  int64_t units;                  // units per group (a unit = one stripe (kind 1/2) or
                                  // one (row group, rest stripe) pair (kind 3)) times ksplit
  int64_t chunk;                  // units per workgroup
  int32_t ksplit;                 // contraction range split into this many pieces
  int32_t kchunk;                 // contraction length per piece (multiple of 16)
  int32_t rgroups;                // kind 3: number of row groups over I1
  int64_t rest_count;             // kind 3: number of stripes per output value
  int32_t prep;                   // 1: workgroup 0 runs sweep_prep(pa) instead of streaming
  int32_t vec;                    // 4-wide tensor loads allowed (I0 % 4 == 0, aligned base)
  double* y;                      // kind 2 with ksplit == 1: also store the stage-1 tiles
                                  // Y[s][i1][r] = sum_i0 Z(i0, i1, s) A^(0)(i0, r), in the
                                  // tensor's precision (FP32 tensor: the FP32 MFMA sums as
                                  // they are, stored as float at y; FP64: doubles)
  PrepArgs pa;
};

// Dimension-tree MTTKRP of a mode n >= 2 from the stored stage-1 tiles Y of the
// mode-1 launch (Y depends only on Z and A^(0), so it serves every mode after 1):
//   M^(n)(i_n, r) = sum_{s : s_n = i_n} sum_i1 Y[s][i1][r] A^(1)(i1, r) prod_{m >= 2, m != n} A^(m)(s_m, r)
struct YDesc {
  const double* y;                // [S][I1][R]; floats when y32
  int32_t y32;
  const double* a64[kMaxOrder];
  double* out;                    // partials [nsplit][I_n][R]
  int64_t I1, S, In;
  int32_t N, n, R;
  int32_t ns;
  int64_t sext[kMaxOrder], sst[kMaxOrder];
  int64_t rest_count;             // stripes per output value (S / I_n)
  int64_t rchunk;                 // rest indices per split
  int32_t nsplit;
  int32_t prep;
  PrepArgs pa;
};
// plan (nsplit) for a mode-n launch from Y, and the launch itself
int ymttkrp_nsplit(const int64_t* dims, int N, int n, int R);
hipError_t ymttkrp_launch(const int64_t* dims, int N, int n, int R, const double* y, bool y32,
                          const double* const* a64, double* out, int nsplit, const PrepArgs* prep,
                          hipStream_t st);

// planner + launcher (mttkrp.hip)
struct PlanOpts {
  int32_t target_wgs;   // streaming workgroups to aim for
  int32_t ksplit;       // pieces of the contraction range (0: automatic)
  int32_t tw;           // 16-row tiles per wave, kinds 2/3 (0: 2)
  int32_t vw;           // FP32: tensor entries per lane load, 4 (16 B) or 8 (32 B)
  int32_t nostage;      // 1: read the contracted factor from global memory instead of
                        //    staging it in LDS at the start of every workgroup
};

struct MttkrpPlan {
  int32_t kind, nsplit, ngroups, ksplit, kchunk, rgroups;
  int64_t chunk, units;
  size_t partial_doubles;   // nsplit * I_n * R
  int32_t tw;               // row tiles per wave (kind 2/3)
  int32_t nt;               // 16-column tiles (ceil(R/16))
  int32_t vw;               // tensor entries per lane load
  int32_t bl;               // 1: the contracted factor is staged in LDS
  int64_t bstage_doubles;   // its LDS footprint (doubles) when bl
  PlanOpts opts;            // options the plan was made from
};

MttkrpPlan mttkrp_plan(int N, const int64_t* dims, int n, int R, bool fp32, const PlanOpts& o);
// resident workgroups of the plan's kernel on the whole device
int mttkrp_capacity(const MttkrpPlan& p, bool fp32);
// y: mode-1 launches with an unsplit contraction may also store Y (dimension tree)
hipError_t mttkrp_launch(const MttkrpPlan& plan, const int64_t* dims, int N, int n, int R,
                         const void* z, bool fp32, const double* const* a64,
                         const float* const* a32, double* out, const PrepArgs* prep,
                         hipStream_t st, double* y = nullptr);
// The launch descriptor mttkrp_launch would use (for batched launches).
MttkrpDesc mttkrp_desc(const MttkrpPlan& plan, const int64_t* dims, int N, int n, int R,
                       const void* z, bool fp32, const double* const* a64,
                       const float* const* a32, double* out, const PrepArgs* prep,
                       double* y = nullptr);
// dynamic LDS bytes of a launch of `plan` (with or without the bookkeeping workgroup)
size_t mttkrp_smem_bytes(const MttkrpPlan& p, int N, int R, bool prep);
// Batched MTTKRPs of one mode: tile t runs workgroup tiles[t].y of descs[tiles[t].x]
// (device arrays; 16-column tiles nt = 1 or 2 for every listed problem, the
// contracted factor staged in LDS, rows per wave 2, 4-wide lanes).
hipError_t mttkrp_batched_launch(int kind, bool fp32, int nt, const MttkrpDesc* descs,
                                 const int2* tiles, int ntiles, size_t smem_bytes, hipStream_t st);

// ---------------------------------------------------------------------------
// Mode epilogue: reduce MTTKRP partials and act on the rows
// ---------------------------------------------------------------------------
enum EpiOp : int32_t {
  EPI_STORE_M = 0,   // M = sum of partials (cp_mttkrp)
  EPI_UPDATE = 1,    // A^(n) <- solve((M + F) , Gamma)  + Gram^(n) + objective pieces
  EPI_GRAD = 2,      // accumulate ||A Gamma - M||^2 into a scalar
  EPI_H = 3,         // H = A Gamma - M (FAS operator) into a buffer
};

struct EpiDesc {
  int32_t op, solver, gs_iters, R, N, n;
  int32_t nsplit;
  int64_t In;
  const double* partial;      // [nsplit][In][R]
  const double* F;            // optional (I_n x R) right-hand side
  double* A;                  // factor n (FP64)
  float* A32;                 // optional shadow
  double* outbuf;             // EPI_STORE_M / EPI_H target
  double* grams;              // [N][R][R]  (Upsilon of each mode)
  const double* prep_out;     // EPI_UPDATE: [R*R + 2R] from sweep_prep
  const int32_t* kind;        // EPI_UPDATE: 0 Cholesky factor, 1 pseudoinverse, 2 Gamma (GS)
  double* scal_part;          // [nwg] workspace (x groups for EPI_UPDATE with want_obj)
  int32_t groups;             // EPI_UPDATE: column groups (0 or 1: one group)
  const BatchState* st;       // EPI_UPDATE in a batched solve: skip frozen groups
  int32_t run_phase;          // ... and problems not in this launch's phase
  int32_t* counter;           // last-block counter (zero between launches)
  double* scalar_out;         // objective: f_hist slot; grad: accumulator
  const double* norm2;        // ||Z||^2 (device)
  uint32_t* flags;
  int32_t want_obj;           // EPI_UPDATE: per-block <A^(n), M^(n)> into scal_part
  int32_t accumulate;         // EPI_GRAD: add to scalar_out instead of overwrite
};

hipError_t epi_launch(const EpiDesc& d, hipStream_t st);
int epi_rows_per_wg();
// batched: tile t runs block tiles[t].y of the epilogue descs[tiles[t].x] (device arrays)
hipError_t epi_batched_launch(const EpiDesc* descs, const int2* tiles, int ntiles, hipStream_t st);

// Batched Gram jobs (one mode of one problem each)
struct GramJob {
  const double* A;
  float* A32;           // refreshed from A when set
  int64_t I;
  int32_t R;
  double* gram;         // R x R output
  double* sigma;        // R column scales reset to 1 when set
  const BatchState* st; // skip when the problem is inactive
};
// one workgroup per (listed problem, mode): jobs[plist[j / N] * N + j % N]
hipError_t gram_batched_launch(const GramJob* jobs, const int32_t* plist, int count, int N,
                               hipStream_t st);

// End of a sweep sequence: Gram of the last mode, fused objective, and the
// pending normalization applied to the stored factors (one workgroup).
hipError_t finalize_launch(const PrepArgs& a, hipStream_t st);
// batched: one workgroup per listed problem (pas[plist[j]], device arrays)
hipError_t finalize_batched_launch(const PrepArgs* pas, const int32_t* plist, int count,
                                   int smem_doubles, hipStream_t st);

// Grams of every mode at fixed A; optionally refresh FP32 shadows and reset the
// pending normalization scales (sigma, N x R) to 1
hipError_t gram_launch(double* const* A, float* const* A32, const int64_t* dims, int N, int R,
                       double* grams, hipStream_t st, double* sigma = nullptr);


// exact residual ||Z - [[A]]||^2 / 2
hipError_t residual_launch(const double* z, const int64_t* dims, int N, int R,
                           const double* const* A, double* part, int32_t* counter, double* f,
                           hipStream_t st);

// fused objective from a Gram set, inner product and norm (one thread)
hipError_t fused_f_launch(const double* grams, int N, int R, const double* inner,
                          const double* norm2, double* f, hipStream_t st);
// g = sqrt(acc)/sqrt(norm2)
hipError_t finish_g_launch(const double* acc, const double* norm2, double* g, hipStream_t st);
hipError_t inner_launch(const double* A, const double* M, int64_t count, double* part,
                        int32_t* counter, double* out, hipStream_t st);

// Relaxation of a small level in one workgroup (small.hip): `nsweeps` BNGS
// sweeps with Gauss-Seidel inner solves and optional right-hand side F, no
// normalization, the tensor resident in LDS.  Used when the tensor, the
// stage-1 tiles and the factors fit in kSmallLdsBytes and R <= 16.
struct SmallDesc {
  const void* z;                  // tensor (double, or float for the mixed form)
  int32_t N, R, nsweeps, gs_iters;
  int64_t dims[kMaxOrder];
  int64_t P;
  double* A[kMaxOrder];
  float* A32[kMaxOrder];          // refreshed at the end when set
  const double* F[kMaxOrder];     // NULL: no right-hand side
};
constexpr size_t kSmallLdsBytes = 152 * 1024;
bool small_eligible(const SmallDesc& d, bool fp32);
size_t small_lds_bytes(const SmallDesc& d, bool fp32);
hipError_t relax_small_launch(const SmallDesc& d, bool fp32, hipStream_t st);

// LS interpolation weights of one mode from the column groups of a factor set
// (setup.hip): A, M (I x Rt), Grams of the set, fitted groups 0..nfit-1 of Rg columns.
hipError_t interp_weights_launch(const double* A, const double* M, const double* grams, int N, int n,
                                 int64_t I, int Rt, int Rg, int nfit, double* w, hipStream_t st);

// Sparse tensors (sparse.hip): coordinate entries with per-mode orderings
// (cp_tensor's sparse form).
struct SpTensor {
  int32_t N;
  int64_t nnz;
  int64_t dims[kMaxOrder];
  const int32_t* idx;                 // [nnz][N]
  const double* vals;                 // [nnz]
  const int64_t* rowptr[kMaxOrder];   // per mode: I_m + 1 offsets into perm[m]
  const int32_t* perm[kMaxOrder];     // per mode: entry ids by (index, id)
};
// MTTKRP of mode n over the stored entries: workgroup (row i, split q) sums
// the q-th share of row i's entries into partials [nsplit][I_n][R]; with a
// bookkeeping workgroup in front when prep != NULL (as the dense launches).
constexpr int32_t kSparseKind = 4;     // MttkrpPlan::kind of a sparse launch
int sp_mttkrp_nsplit(const SpTensor& t, int n);
hipError_t sp_mttkrp_launch(const SpTensor& t, int n, int R, const double* const* a64, double* out,
                            int nsplit, const PrepArgs* prep, hipStream_t st);
// dense[lin(idx_k)] = vals[k] (dense must hold zeros elsewhere)
hipError_t sp_densify_launch(const SpTensor& t, double* dense, hipStream_t st);
// host: per-mode orderings of the entries (cp_sparse_index); returns an error
// code and message for bad input
cp_status sparse_index_host(int order, const int64_t* dims, int64_t nnz, const int32_t* idx,
                            int64_t* rowptr, int32_t* perm, std::string* msg);

// utilities
hipError_t cast_launch(const double* src, float* dst, int64_t count, hipStream_t st);
hipError_t norm2_launch(const double* z, int64_t count, double* part, int32_t* counter,
                        double* out, hipStream_t st);
hipError_t fill_launch(double* dst, double v, int64_t count, hipStream_t st);
hipError_t copy_launch(const double* src, double* dst, int64_t count, hipStream_t st);

// transfer operators (transfer.hip)
hipError_t transfer_build_launch(int64_t I, const double* w, double* phat, double* ws /*2*Ic*/,
                                 hipStream_t st);
hipError_t prolong_launch(int64_t I, int64_t Ic, int R, const double* phat, const double* Ac,
                          const double* Act, double* A, hipStream_t st);
hipError_t restrict_factor_launch(int64_t I, int64_t Ic, int R, const double* phat,
                                  const double* A, double* Ac, hipStream_t st);
// factored restriction (transfer.hip): coefficients of every coarsened mode
// from its interpolation weights (one launch), then per mode the stencil +
// bidiagonal solve over a tensor viewed as (Lead, I, Tail)
struct RCoefJobs {                 // one entry per coarsened mode
  int32_t count;
  int64_t I[kMaxOrder];
  const double* w[kMaxOrder];
  void* coef[kMaxOrder];           // 4 Ic doubles
  double* scratch[kMaxOrder];      // 2 Ic doubles
};
hipError_t restrict_coef_launch(const RCoefJobs& jobs, hipStream_t st);
hipError_t restrict_factored_launch(const void* in, void* out, int64_t Lead, int64_t I, int64_t Tail,
                                    const void* coef, bool fp32, hipStream_t st);
// Fc = Hc + P^^T (F - H)   (F may be NULL = 0)
hipError_t fas_rhs_launch(int64_t I, int64_t Ic, int R, const double* phat, const double* F,
                          const double* H, const double* Hc, double* Fc, hipStream_t st);
// Fc = F - H + Hc (tau rule, identity transfer) or Fc = F (literal)
hipError_t fas_rhs_identity_launch(int64_t count, const double* F, const double* H,
                                   const double* Hc, int literal, double* Fc, hipStream_t st);

// batched strided GEMM on the matrix cores: C[b] = A[b] * B[b]
struct GemmDesc {
  const void* A; const void* B; void* C;
  int64_t M, N, K, batch;
  int64_t a_rs, a_cs, a_bs;
  int64_t b_rs, b_cs, b_bs;
  int64_t c_rs, c_cs, c_bs;
};
hipError_t gemm_launch(const GemmDesc& d, bool fp32, hipStream_t st);

hipError_t sort_launch(double* const* A, float* const* A32, const int64_t* dims, int N, int R,
                       double* scratch, hipStream_t st);

}  // namespace cpamg

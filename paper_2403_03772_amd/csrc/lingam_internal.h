// Internal interface between the C ABI (lingam_abi.cpp) and the gfx950
// kernels (lingam_kernels.hip).  Not installed; not part of the ABI.
//
// Every ordering runs as a batch of jobs (a single ordering is a batch of
// one).  Each job has its own workspace regions; a device-resident job table
// (JobDev) carries their addresses, and every step kernel covers the current
// step of all active jobs: a small schedule kernel writes, per job, the step's
// plan (JobStep) and exclusive prefix sums of each kernel's workgroup counts;
// a workgroup finds its job by binary search over those sums.  The host
// replays the same plan arithmetic (the functions below are __host__
// __device__) to size the grids, so the whole ordering is enqueued without any
// host synchronisation and can be captured into one HIP graph.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lg {

// Variables per side of a pair tile handled by one workgroup (2 x 2 waves of
// 4 x 4 variables each).
constexpr int kTileVars = 8;
constexpr int kWaveVars = 4;
// Samples are padded to a multiple of this (one wavefront of samples).
constexpr int kSampleQuantum = 64;
// Steps with at most this many active variables run the FP64 pair kernel.
constexpr int kFp64MaxM = 64;
// Most aggressive split policy the workspace is sized for (see Tune).
constexpr int kMaxTargetPerCu = 32;
constexpr int kMinMinIters = 4;

// Device control block (one per job, in the workspace).
struct Ctrl {
  int32_t status;    // 0 = ok, else a negative lingam_status
  int32_t exo_slot;  // original id chosen at the current step
  int32_t exo_pos;   // its position in the active list before removal
  int32_t pad[61];
};

// Byte offsets of one job's workspace regions.
struct Layout {
  int64_t n, d, n_pad, ldz;  // ldz = n_pad elements per variable row
  size_t zd;     // double [(d + 1) * ldz]  variable-major residuals, row d = zeros
  size_t z;      // float  [(d + 1) * ldz]  FP32 copy read by the pair kernel
  size_t mu;     // double [d]
  size_t sig;    // double [d]
  size_t rho;    // double [d * d]  correlation of the current residuals, by original id
  size_t hm;     // double [d]      marginal entropy H(z_v), by original id
  size_t act;    // int32  [d]      active list (original ids by position)
  size_t ctrl;   // Ctrl
  size_t part;   // double [part_elems] pair-kernel partial sums
  size_t rmat;   // double [d * d]  pairwise measure R by position
  size_t mvec;   // double [d]      per-position measure -k
  size_t total;
  size_t part_elems;
};

// Device job table entry (absolute device addresses).
struct JobDev {
  const float* X;        // FP32 row-major samples, or NULL when Zd is pre-filled
  const int32_t* rows;   // optional sample -> row map (bootstrap resampling)
  int64_t ldx;
  int32_t n, d, n_pad, ldz;
  int32_t* order;        // [d]
  double* measures;      // [(d-1) * d] or NULL
  double* gaps;          // [d-1] or NULL
  const int32_t* forced;
  int32_t forced_len, n_src;  // n_src: rows of X (bounds of `rows`)
  double* zd;
  float* z;
  double* mu;
  double* sig;
  double* rho;
  double* hm;
  int32_t* act;
  Ctrl* ctrl;
  double* part;
  double* rmat;
  double* mvec;
};

// Split policy of the pair kernel (autotuned): enough workgroups for
// target_per_cu per CU, at least min_iters sample iterations per split.
struct Tune {
  int32_t target_per_cu;
  int32_t min_iters;
};

// One job's plan for one step.
struct JobStep {
  int32_t m;          // active variables (0: job finished before this step)
  int32_t nblk;       // ceil(m / kTileVars)
  int32_t ntiles;     // nblk (nblk + 1) / 2
  int32_t nsplit;     // sample splits per (tile, direction)
  int32_t split_len;  // samples per split
  int32_t fp64;       // 1: FP64 pair path (m <= kFp64MaxM)
};

// Workgroup-count kinds with a prefix array each.
enum Kind : int {
  kKPair = 0,   // k_pair: ntiles * 2 * nsplit
  kKComb,       // k_combine: ceil(ntiles / 4)
  kKP64,        // k_pair64: ceil(m (m - 1) / 2 / 4)
  kKRowk,       // k_rowk: ceil(m / 4)
  kKSel,        // k_select: 1
  kKRes,        // k_resid: m - 1 when m > 2
  kNumKinds
};
// Set-up kinds (one schedule before the first step).
enum SetupKind : int {
  kSIngest = 0,  // (n_pad / 64) * ceil((d + 1) / 64)
  kSCols,        // d (moments, standardize)
  kSGram,        // nb (nb + 1) / 2, nb = ceil(d / 32)
  kNumSetupKinds
};

__host__ __device__ inline int32_t cdiv(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

// The step's plan for a job without the split (needs the batch-wide sum).
__host__ __device__ inline JobStep job_step_base(int32_t d, int32_t t) {
  JobStep s{};
  const int32_t m = d - t;
  if (m < 2) return s;
  s.m = m;
  s.fp64 = m <= kFp64MaxM;
  if (!s.fp64) {
    s.nblk = cdiv(m, kTileVars);
    s.ntiles = s.nblk * (s.nblk + 1) / 2;
  }
  return s;
}

// Split of one FP32-path job given the batch's number of (tile, direction) items.
__host__ __device__ inline void job_split(JobStep& s, int32_t n_pad, int64_t items_total,
                                          int32_t num_cu, Tune tu) {
  if (s.m < 2 || s.fp64) return;
  const int64_t iters = n_pad / kSampleQuantum;
  const int64_t target = (int64_t)num_cu * tu.target_per_cu;
  int64_t ns = items_total > 0 ? (target + items_total - 1) / items_total : 1;
  const int64_t cap = iters >= tu.min_iters ? iters / tu.min_iters : 1;
  if (ns > cap) ns = cap;
  if (ns < 1) ns = 1;
  const int64_t per = (iters + ns - 1) / ns;
  s.split_len = (int32_t)(per * kSampleQuantum);
  s.nsplit = (int32_t)((iters + per - 1) / per);
}

__host__ __device__ inline int32_t kind_count(const JobStep& s, int kind) {
  if (s.m < 2) return 0;
  switch (kind) {
    case kKPair: return s.fp64 ? 0 : s.ntiles * 2 * s.nsplit;
    case kKComb: return s.fp64 ? 0 : cdiv(s.ntiles, 4);
    case kKP64: return s.fp64 ? cdiv((int64_t)s.m * (s.m - 1) / 2, 4) : 0;
    case kKRowk: return cdiv(s.m, 4);
    case kKSel: return 1;
    case kKRes: return s.m > 2 ? s.m - 1 : 0;
    default: return 0;
  }
}

__host__ __device__ inline int32_t setup_count(int32_t n_pad, int32_t d, int kind) {
  switch (kind) {
    case kSIngest: return (n_pad / 64) * cdiv(d + 1, 64);
    case kSCols: return d;
    case kSGram: {
      const int32_t nb = cdiv(d, 32);
      return nb * (nb + 1) / 2;
    }
    default: return 0;
  }
}

Layout make_layout(int64_t n, int64_t d, int num_cu);

// Schedule buffer of a batch (device): per step, JobStep[njobs] and
// kNumKinds prefix arrays of njobs + 1 entries; for the set-up,
// kNumSetupKinds prefix arrays.
struct SchedDev {
  JobStep* js;
  int32_t* pre;   // [kNumKinds][njobs + 1]
  int32_t* spre;  // [kNumSetupKinds][njobs + 1]
};
size_t sched_bytes(int njobs);
SchedDev sched_at(char* base, int njobs);

// Kernel launchers (all asynchronous on `st`).  `grid` is the host's total of
// the matching prefix array.
hipError_t launch_setup_schedule(const JobDev* jobs, int njobs, SchedDev sc, hipStream_t st);
hipError_t launch_init(const JobDev* jobs, int njobs, hipStream_t st);
hipError_t launch_ingest(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st);
hipError_t launch_moments(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st);
hipError_t launch_gram(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st);
hipError_t launch_standardize(const JobDev* jobs, int njobs, SchedDev sc, int grid,
                              hipStream_t st);
hipError_t launch_step_schedule(const JobDev* jobs, int njobs, int t, int num_cu, Tune tu,
                                SchedDev sc, hipStream_t st);
hipError_t launch_pair(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st);
hipError_t launch_combine(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st);
hipError_t launch_pair64(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st);
hipError_t launch_rowk(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st);
hipError_t launch_select(const JobDev* jobs, int njobs, int t, SchedDev sc, int grid,
                         hipStream_t st);
hipError_t launch_resid(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st);
hipError_t launch_gather_status(const JobDev* jobs, int njobs, int32_t* dst, hipStream_t st);
// Writes `count` (at most kJobsPerLaunch) job-table entries from kernel arguments.
constexpr int kJobsPerLaunch = 16;
hipError_t launch_set_jobs(JobDev* table, int first, const JobDev* host_jobs, int count,
                           hipStream_t st);

// VarLiNGAM: the ordering layout for the residuals (n = T - lags) followed by
// the VAR regions.
struct VarLayout {
  int64_t T, d, N, p, q, ldx;  // N = T - lags rows, p = 1 + lags d regressors, q = p + d
  int lags;
  Layout ord;    // ordering of the residuals (offsets relative to the job's base)
  // VAR block (offsets relative to its own base)
  size_t xd;     // double [(d + 1) * ldx] the series, variable-major
  size_t ones;   // double [N]
  size_t w;      // double [q * q] Gram of [1, lags, response]; Cholesky + solution in place
  size_t rho0;   // double [d * d] residual correlations before the ordering
  size_t scr;    // double [d * d] scratch of the B0 factorisation
  size_t total;
};

VarLayout make_var_layout(int64_t T, int64_t d, int lags, int num_cu);
// `ws` is the VAR block, `job` the base of the ordering job's regions.
hipError_t launch_var_fit(const VarLayout& V, char* ws, char* job, const float* X, int64_t ldx,
                          float* resid_out, double* M_out, hipStream_t st);
hipError_t launch_save_rho(const VarLayout& V, char* ws, char* job, hipStream_t st);
hipError_t launch_b0(const VarLayout& V, char* ws, char* job, const int32_t* order, double* B0,
                     hipStream_t st);

// Standalone residualisation on a row-major matrix.
size_t resid_ws_size(int64_t n, int64_t d);
hipError_t launch_residualize_rowmajor(float* X, int64_t n, int64_t d, int64_t ldx,
                                       const int32_t* active, int32_t n_active, int32_t exo,
                                       char* ws, hipStream_t st);

}  // namespace lg

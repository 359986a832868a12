// Internal interface between the C ABI (lingam_abi.cpp) and the gfx950
// kernels (lingam_kernels.hip).  Not installed; not part of the ABI.
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

// Device control block (one per call, in the workspace).
struct Ctrl {
  int32_t status;    // 0 = ok, else a negative lingam_status
  int32_t exo_slot;  // original id chosen at the current step
  int32_t exo_pos;   // its position in the active list before removal
  int32_t pad[61];
};

// Byte offsets of the workspace regions of lingam_causal_order.
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

struct StepPlan {
  int nblk;       // ceil(m / kTileVars)
  int ntiles;     // nblk * (nblk + 1) / 2 upper-triangular tiles
  int nsplit;     // sample splits per tile
  int split_len;  // samples per split (multiple of kSampleQuantum)
};

StepPlan plan_step(int64_t m, int64_t n_pad, int num_cu);
Layout make_layout(int64_t n, int64_t d, int num_cu);

// Kernel launchers (all asynchronous on `st`).
hipError_t launch_init(const Layout& L, char* ws, int32_t* order, hipStream_t st);
hipError_t launch_ingest(const Layout& L, char* ws, const float* X, int64_t ldx, hipStream_t st);
hipError_t launch_moments(const Layout& L, char* ws, hipStream_t st);
hipError_t launch_gram(const Layout& L, char* ws, hipStream_t st);
hipError_t launch_standardize(const Layout& L, char* ws, hipStream_t st);
hipError_t launch_pair(const Layout& L, char* ws, int m, const StepPlan& p, hipStream_t st);
hipError_t launch_combine(const Layout& L, char* ws, int m, const StepPlan& p, hipStream_t st);
hipError_t launch_pair64(const Layout& L, char* ws, int m, hipStream_t st);
hipError_t launch_rowk(const Layout& L, char* ws, int m, hipStream_t st);
hipError_t launch_select(const Layout& L, char* ws, int m, int t, int32_t* order,
                         const int32_t* forced, int forced_len, double* step_measures,
                         double* step_gap, hipStream_t st);
hipError_t launch_resid(const Layout& L, char* ws, int m_after, hipStream_t st);
hipError_t launch_copy_status(const Layout& L, char* ws, int32_t* dst, hipStream_t st);

// Standalone residualisation on a row-major matrix.
size_t resid_ws_size(int64_t n, int64_t d);
hipError_t launch_residualize_rowmajor(float* X, int64_t n, int64_t d, int64_t ldx,
                                       const int32_t* active, int32_t n_active, int32_t exo,
                                       char* ws, hipStream_t st);

}  // namespace lg

// Dense FP64 pieces of the library beyond the ordering engine: the
// adaptive-lasso pruning of the adjacency matrix (internal; not installed).
#pragma once

#include "lingam_internal.h"

namespace lg {

// Most active predictors of a pruning path (the LDS inverse is this square).
constexpr int kLassoMaxActive = 64;

// Workspace of lingam_adjacency_pruned: one region set per call.
struct PruneLayout {
  int64_t n, d, ldx;  // ldx = n rounded up to 64
  size_t ctrl;   // Ctrl (status only)
  size_t mark;   // int32  [d]   permutation check
  size_t tol;    // double       pivot tolerance
  size_t mu;     // double [d]   column means
  size_t sd;     // double [d]   standard deviations by position
  size_t xd;     // double [(d + 1) * ldx] the data, variable-major
  size_t s;      // double [d * d] covariance by position
  size_t r;      // double [d * d] correlation by position
  size_t l;      // double [d * d] its Cholesky factor (lower)
  size_t y;      // double [d * d] inverse of the factor
  size_t st;     // double [d * 4 d] path state of every target
  size_t total;
};

PruneLayout make_prune_layout(int64_t n, int64_t d);

// Workspace of lingam_total_effects.
struct EffectsLayout {
  int64_t d;
  size_t ctrl;   // Ctrl (status only)
  size_t mark;   // int32  [d]   permutation check
  size_t a;      // double [d * d] I - B permuted into the order (unit lower)
  size_t x;      // double [d * d] its inverse
  size_t total;
};
EffectsLayout make_effects_layout(int64_t d);
// T = (I - B)^-1 through the order (after the permutation check).
hipError_t launch_total_effects(const EffectsLayout& A, char* ws, const double* B,
                                const int32_t* order, double* T, hipStream_t st);
// After the permutation / row check of launch_adj_check (run on an AdjLayout
// view of the same ctrl and mark regions): B (d x d, row-major) = the pruned
// adjacency.  Status kDegenerate on non-finite data or a correlation matrix
// that is not positive definite.
hipError_t launch_adjacency_pruned(const PruneLayout& A, char* ws, const float* X, int64_t ldx,
                                   const int32_t* rows, const int32_t* order, int max_active,
                                   double* B, hipStream_t st);

}  // namespace lg

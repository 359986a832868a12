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

// Device address of this device's scratch array (lingam_noalloc.hip), looked
// up on the first call per device with that device current, then cached.
hipError_t noalloc_scratch(int dev, void** ptr);

// Variables per side of a pair tile handled by one workgroup (2 x 2 waves of
// 4 x 4 variables each).
constexpr int kTileVars = 8;
constexpr int kWaveVars = 4;
// Samples are padded to a multiple of this (one wavefront of samples).
constexpr int kSampleQuantum = 64;
// Resident waves per CU of the pair kernels (their register budget allows 5
// waves per SIMD): the bounded grids of the gated full step and of the
// suspect and extension passes launch kPairWavesPerCu / w workgroups of w
// waves per CU.
constexpr int kPairWavesPerCu = 16;
// Steps with at most this many active variables run the FP64 pair kernel.
constexpr int kFp64MaxM = 64;
// Most aggressive split policy the workspace is sized for (see Tune).
constexpr int kMaxTargetPerCu = 32;
constexpr int kMinMinIters = 4;

// Learned-proposal form: a 16 -> 128 -> 128 -> 1 ReLU network scores every
// active variable, the exact measure is evaluated for the kTopK best.
constexpr int kFeat = 16;
constexpr int kHidden = 128;
constexpr int kParams = kHidden * kFeat + kHidden + kHidden * kHidden + kHidden + kHidden + 1;
constexpr int kPropNorm = 2 * kFeat;  // feature mean and scale ahead of the weights
constexpr int kMaxTopK = 256;
// Most suspects (non-candidates whose lower bound does not exceed the best
// candidate's k) a second candidate pass evaluates in one step.
constexpr int kMaxSuspects = 1024;
// Witnesses per variable: the most correlated other active variables, whose
// pair measures join the candidates' in a learned step's lower bound on k.
constexpr int kWit = 8;
// FP64 tie resolution.  The FP32 pair kernels measure k to about 1e-3 of its
// own value at the noise level of the largest workloads, so when the best k
// of a step and others lie within tie_limit of each other (at most kMaxTie
// of them), the step's choice is made from their rows recomputed in FP64
// (the FP64 residuals, correlations and marginal entropies the step already
// holds) instead of from the FP32 values.
constexpr int kMaxTie = 16;
constexpr double kTieRel = 4e-3;
constexpr double kTieAbs = 1e-12;
__host__ __device__ inline double tie_limit(double kbest) {
  return kbest * (1.0 + kTieRel) + kTieAbs;
}
// Most extension columns: the variables ranked right after the candidates,
// measured against the suspects before their full rows are.
constexpr int kMaxExt = 256;
// offsets of the trainable parameters inside the flat FP32 block
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHidden * kFeat;
constexpr int kOffW2 = kOffB1 + kHidden;
constexpr int kOffB2 = kOffW2 + kHidden * kHidden;
constexpr int kOffW3 = kOffB2 + kHidden;
constexpr int kOffB3 = kOffW3 + kHidden;

// Device copy of the network for one run (BF16 weights, FP32 biases).
struct PropDev {
  uint16_t w1[kHidden * kFeat];    // W1[h][f]
  uint16_t w2[kHidden * kHidden];  // W2[h][g]
  uint16_t w3[kHidden];
  float b1[kHidden];
  float b2[kHidden];
  float mu[kFeat];
  float sd[kFeat];
  float b3;
  float pad[63];
};

// Device control block (one per job, in the workspace).
struct Ctrl {
  int32_t status;    // 0 = ok, else a negative lingam_status
  int32_t exo_slot;  // original id chosen at the current step
  int32_t exo_pos;   // its position in the active list before removal
  int32_t full;      // learned step: 1 = the full step decides
  int32_t learned_slot;  // learned step: the best candidate's original id
  int32_t n_learned;     // learned steps taken
  int32_t n_certified;   // ... of which certified exact
  int32_t n_fallback;    // full steps taken because the margin was small
  int32_t n_audit;       // audit steps
  int32_t n_audit_agree; // audits whose full choice equalled the learned one
  float s_out;           // best score outside the candidates (this step)
  int32_t n_suspects_max;  // largest count of non-candidates whose bound <= k_best
  long long n_suspects_sum;
  int32_t nsus;            // this step: suspects listed for the second pass (0: none)
  int32_t n_expanded;      // learned steps decided exactly by the second pass
  int32_t n_cleared;       // ... of which every suspect was cleared by the extension columns
  long long n_rows_sum;    // suspects whose full rows the second pass measured
  int32_t ntie;            // near-tied positions listed for the FP64 decision of
  int32_t tie_t;           // ... step tie_t (at any other step: none pending)
  int32_t tie_audit;       // 1: the deferred decision is an audit step's full step
  int32_t n_ties;          // steps decided by the FP64 tie resolution
  int32_t n_tie_rows;      // ... rows they measured in FP64
  int32_t tie_done;        // rows of the FP64 decision finished
  int32_t n_tie_overflow;  // steps with more than kMaxTie near-tied positions (the
                           // FP32 measures decided them)
  int32_t tie_row_done[kMaxTie];  // pairs of each row of the FP64 decision finished
  int32_t pad[21];
};
static_assert(sizeof(Ctrl) == 256, "control block is 256 bytes");

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
  size_t mom;    // double [d * 8]  moments of z by original id (E lc, E g, E z^3, E z^4, E|z|)
  // learned form (K > 0 only)
  int32_t K;
  size_t feat;   // float  [d * kFeat] features by position
  size_t score;  // float  [d]      network score by position
  size_t cand;   // int32  [kMaxTopK] candidate positions (ascending)
  size_t cmark;  // int32  [d]      t + 1 at candidate positions of step t
  size_t partc;  // double [partc_elems] candidate pair-kernel partial sums
  size_t rc;     // double [K * d]  R(candidate, position)
  size_t kc;     // double [K]      exact k of every candidate
  size_t lb;     // double [d]      lower bound of k at excluded positions
  size_t wit;    // int32  [d * kWit] witness positions of every position (-1: none)
  size_t ext;    // int32  [kMaxExt] extension positions (ascending; padding = m)
  size_t steplog;  // int32 [d]     per step: 0 plain, 1 learned, 2 fallback, 3 audit
  // second candidate pass over the suspects
  int32_t cap_s;   // most suspects listed (kMaxSuspects or less, multiple of 8)
  size_t cand2;    // int32  [cap_s] suspect positions (ascending; padding = m)
  size_t parts;    // double [parts_elems] partial sums
  size_t rc2;      // double [cap_s * d] R(suspect, position)
  size_t kc2;      // double [cap_s] exact k of every suspect
  // FP64 tie resolution (every job)
  size_t tie;      // int32  [kMaxTie] near-tied positions of the current step
  size_t tie_r;    // double [kMaxTie * d] their FP64 measure rows, then their k [kMaxTie]
  size_t total;
  size_t part_elems;
  size_t partc_elems;
  size_t parts_elems;
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
  double* mom;
  // learned form
  const PropDev* prop;   // NULL: plain search
  int32_t K, min_m, audit_every;
  float delta;
  float* record;         // optional [(d - 1) * d * kFeat] features by step and original id
  float* feat;
  float* score;
  int32_t* cand;
  int32_t* cmark;
  double* partc;
  double* rc;
  double* kc;
  double* lb;
  int32_t* wit;
  int32_t* ext;
  int32_t ne_max;        // extension columns per learned step (0: none)
  int32_t* steplog;
  int32_t cap_s;
  int32_t* cand2;
  double* parts;
  double* rc2;
  double* kc2;
  // FP64 tie resolution
  int32_t tie_on;        // 1: near-ties are decided in FP64
  int32_t* tie;
  double* tie_r;
};

// Launch shape of the pair kernels (autotuned).
//   Split policy of the sample range: enough (tile, direction) items for
//   target_per_cu workgroups per CU, at least min_iters sample iterations per
//   split.  The split decides which samples each lane sums, so it changes
//   results at the rounding level.
//   Waves per workgroup of the all-pairs kernel (w_all) and of the learned
//   form's row kernels (w_rows), 1, 2 or 4: a workgroup takes w of the four
//   4 x 4 quadrants of an 8 x 8 tile.  Every wave sums exactly what it sums
//   in any other shape, so the results do not depend on these two.
struct Tune {
  int32_t target_per_cu;
  int32_t min_iters;
  int32_t w_all;
  int32_t w_rows;
};
__host__ __device__ inline bool valid_waves(int32_t w) { return w == 1 || w == 2 || w == 4; }

// One job's plan for one step.
struct JobStep {
  int32_t m;          // active variables (0: job finished before this step)
  int32_t nblk;       // ceil(m / kTileVars)
  int32_t ntiles;     // nblk (nblk + 1) / 2
  int32_t nsplit;     // sample splits per (tile, direction)
  int32_t split_len;  // samples per split
  int32_t fp64;       // 1: FP64 pair path (m <= kFp64MaxM)
  int32_t feat;       // 1: features are computed this step
  int32_t learned;    // 1: learned pass this step (m > min_m)
  int32_t gate;       // 1: the full step is skipped (set after the learned decision)
  int32_t nct;        // candidate tiles (K / 8) * nblk
  int32_t nsplit_c;   // sample splits of the candidate-row kernel
  int32_t split_len_c;
  int32_t nsplit_s;   // ... of the suspect-row kernel (set with the suspect plan)
  int32_t split_len_s;
  int32_t nsus;       // suspects of the second pass (set after the learned decision)
  int32_t nct2;       // suspect tiles ceil(nsus / 8) * nblk
  int32_t k;          // candidates of this step's learned pass
  int32_t ne;         // extension columns (set with the suspect plan)
  int32_t nct3;       // extension tiles ceil(nsus / 8) * ceil(ne / 8)
  int32_t q_all;      // workgroups per tile item of the all-pairs kernel (4 / w_all)
  int32_t q_rows;     // ... of the learned row kernels (4 / w_rows)
};

// Candidates of a learned step with m active variables and at most K: about
// m / 16 (a multiple of 8), at least min(32, K) and at most K.
__host__ __device__ inline int32_t step_topk(int32_t m, int32_t K) {
  const int32_t lo = K < 32 ? K : 32;
  int32_t k = (m / 16 + kTileVars - 1) / kTileVars * kTileVars;
  k = k < lo ? lo : k;
  return k > K ? K : k;
}

// Workgroup-count kinds with a prefix array each.
enum Kind : int {
  kKPair = 0,   // k_pair: ntiles * 2 * nsplit * q_all
  kKComb,       // k_combine: ceil(ntiles / 4)
  kKP64,        // k_pair64: ceil(m (m - 1) / 2 / 4)
  kKRowk,       // k_rowk: ceil(m / 4)
  kKSel,        // k_select: 1
  kKRes,        // k_resid: m - 1 when m > 2
  kKFeat,       // k_features: ceil(m / 4)
  kKMlp,        // k_mlp: ceil(m / 16)
  kKTopk,       // k_topk: 1
  kKPairC,      // k_pair_cand: nct * 2 * nsplit_c * q_rows
  kKCombC,      // k_combine_cand: ceil(nct / 4)
  kKRowkC,      // k_cand_k rows: K / 4
  kKColC,       // k_cand_k columns: ceil(m / 64)
  kKLsel,       // k_lselect: 1
  kKWit,        // k_pair_wit: m
  kKPairE,      // k_pair_ext: nct3 * 2 * nsplit * q_rows (after the learned decision)
  kKBoundE,     // k_ext_bound: ceil(nsus / 4) when nct3 > 0
  kKCompE,      // k_ext_compact: 1 when nct3 > 0
  kKPairS,      // k_pair_susp: nct2 * 2 * nsplit_s * q_rows (after the learned decision)
  kKCombS,      // k_combine_susp: ceil(nct2 / 4)
  kKRowkS,      // k_susp_rowk: ceil(nsus / 4)
  kKLsel2,      // k_lselect2: 1 when nsus > 0
  kNumKinds
};
// the full-step kinds a learned decision can gate off
__host__ __device__ inline bool gated_kind(int kind) {
  return kind == kKPair || kind == kKComb || kind == kKP64 || kind == kKRowk || kind == kKSel;
}
// Set-up kinds (one schedule before the first step).
enum SetupKind : int {
  kSIngest = 0,  // (n_pad / 64) * ceil((d + 1) / 64)
  kSCols,        // d (moments, standardize)
  kSGram,        // nb (nb + 1) / 2, nb = ceil(d / 32)
  kNumSetupKinds
};

__host__ __device__ inline int32_t cdiv(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

// Tile order of the all-pairs kernel: the upper triangle of nb x nb blocks
// (bi <= bj) is walked in super-blocks of kSuperTile x kSuperTile blocks --
// super-rows in order; in each, the diagonal triangle, then the full-height
// blocks to its right -- so the tiles that run at the same time on one XCD
// read few distinct rows.  Bijective from [0, nb (nb + 1) / 2).
constexpr int kSuperTile = 8;
// 32-bit unsigned arithmetic throughout (tile counts are int32, so every
// intermediate below stays under 2^32), with shifts where the super-row and
// the block are full (height and width kSuperTile): in a kernel's prologue a
// 64-bit division is over a hundred scalar instructions.
__host__ __device__ inline void decode_tile_st(int tile, int nb, int& bi, int& bj) {
  constexpr uint32_t S = kSuperTile;
  static_assert(S == 8, "the shifts below assume 8 x 8 super-blocks");
  const uint32_t t = (uint32_t)tile, B = (uint32_t)nb;
  const uint32_t ns = (B + S - 1) / S;
  // tiles before full super-row q: q S (S + 1) / 2 + S (q nb - S q (q + 1) / 2)
  auto pre = [B](uint32_t q) -> uint32_t {
    return q * (S * (S + 1) / 2) + S * (q * B - S * (q * (q + 1) / 2));
  };
  uint32_t lo = 0, hi = ns - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (pre(mid) <= t) lo = mid;
    else hi = mid - 1;
  }
  const uint32_t r0 = lo * S;
  const uint32_t h = B - r0 < S ? B - r0 : S;
  uint32_t r = t - pre(lo);
  const uint32_t diag = h * (h + 1) / 2;
  if (r < diag) {
    uint32_t a = 0;
    while (r >= h - a) {
      r -= h - a;
      ++a;
    }
    bi = (int)(r0 + a);
    bj = (int)(r0 + a + r);
    return;
  }
  r -= diag;
  const uint32_t hs = h * S;
  const uint32_t blk = h == S ? r >> 6 : r / hs;
  const uint32_t rem = r - blk * hs;
  const uint32_t c0 = r0 + S * (blk + 1);
  const uint32_t w = B - c0 < S ? B - c0 : S;
  bi = (int)(r0 + (w == S ? rem >> 3 : rem / w));
  bj = (int)(c0 + (w == S ? rem & 7u : rem % w));
}

// The step's plan for a job without the split (needs the batch-wide sum).
// K > 0 and m > min_m: learned pass; rec: features are recorded every step.
__host__ __device__ inline JobStep job_step_base(int32_t d, int32_t t, int32_t K = 0,
                                                 int32_t min_m = 0, bool rec = false) {
  JobStep s{};
  const int32_t m = d - t;
  if (m < 2) return s;
  s.m = m;
  s.fp64 = m <= kFp64MaxM;
  if (!s.fp64) {
    s.nblk = cdiv(m, kTileVars);
    s.ntiles = s.nblk * (s.nblk + 1) / 2;
  }
  s.learned = K > 0 && m > min_m && !s.fp64;
  s.feat = s.learned || rec;
  if (s.learned) {
    s.k = step_topk(m, K);
    s.nct = (s.k / kTileVars) * s.nblk;
  }
  return s;
}

// Sample split of a pair pass with `items_total` (tile, direction) items over
// the batch: enough splits for about target_per_cu items per CU, each at
// least min_iters 64-sample blocks long.
__host__ __device__ inline void split_for(int64_t items_total, int32_t n_pad, int32_t num_cu,
                                          Tune tu, int32_t& nsplit, int32_t& split_len) {
  const int64_t iters = n_pad / kSampleQuantum;
  const int64_t target = (int64_t)num_cu * tu.target_per_cu;
  int64_t ns = items_total > 0 ? (target + items_total - 1) / items_total : 1;
  const int64_t cap = iters >= tu.min_iters ? iters / tu.min_iters : 1;
  if (ns > cap) ns = cap;
  if (ns < 1) ns = 1;
  const int64_t per = (iters + ns - 1) / ns;
  split_len = (int32_t)(per * kSampleQuantum);
  nsplit = (int32_t)((iters + per - 1) / per);
}

// Split of one FP32-path job given the batch's number of (tile, direction) items.
__host__ __device__ inline void job_split(JobStep& s, int32_t n_pad, int64_t items_total,
                                          int32_t num_cu, Tune tu) {
  s.q_all = valid_waves(tu.w_all) ? 4 / tu.w_all : 1;
  s.q_rows = valid_waves(tu.w_rows) ? 4 / tu.w_rows : 1;
  if (s.m < 2 || s.fp64) return;
  split_for(items_total, n_pad, num_cu, tu, s.nsplit, s.split_len);
}

// Extension columns of a learned step: the next ne_max ranks after the K
// candidates, as many as there are.
__host__ __device__ inline int32_t ext_count(int32_t m, int32_t K, int32_t ne_max) {
  const int32_t r = m - K;
  return r < ne_max ? (r > 0 ? r : 0) : ne_max;
}

// Most suspects a job with m active variables and K candidates lists: the
// second pass must cost less than the full step (2 (K + S) < m rows), and at
// most cap_s (the layout's room); a multiple of 8.
__host__ __device__ inline int32_t suspect_cap(int32_t m, int32_t K, int32_t cap_s) {
  int32_t c = m / 2 - K;
  c = c < cap_s ? c : cap_s;
  return c > 0 ? c / 8 * 8 : 0;
}

// Split of the candidate-row pass (job_split first): its own, from the
// batch's candidate items, so that a pass of a few rows still fills the
// device.  Its measures then differ from the full step's by FP32 rounding,
// and the exact mode's decisions rest on the FP64 resolution of every step
// whose best measures lie within that rounding (tie_limit).  Without that
// resolution (`own` false) the pass takes the full step's split, so that it
// measures every pair bit for bit as the full step does.  The extension
// pass always takes the full step's split.
__host__ __device__ inline void job_split_cand(JobStep& s, int32_t n_pad, int64_t items_c,
                                               int32_t num_cu, Tune tu, bool own) {
  if (!s.learned) return;
  if (own) {
    split_for(items_c, n_pad, num_cu, tu, s.nsplit_c, s.split_len_c);
  } else {
    s.nsplit_c = s.nsplit;
    s.split_len_c = s.split_len;
  }
}

// Split of the suspect-row pass, set with the suspect plan (the same rule
// on the batch's suspect items).
__host__ __device__ inline void job_split_susp(JobStep& s, int32_t n_pad, int64_t items_s,
                                               int32_t num_cu, Tune tu, bool own) {
  if (own) {
    split_for(items_s, n_pad, num_cu, tu, s.nsplit_s, s.split_len_s);
  } else {
    s.nsplit_s = s.nsplit;
    s.split_len_s = s.split_len;
  }
}

__host__ __device__ inline int32_t kind_count(const JobStep& s, int kind) {
  if (s.m < 2) return 0;
  if (s.gate && gated_kind(kind)) return 0;
  switch (kind) {
    case kKPair: return s.fp64 ? 0 : s.ntiles * 2 * s.nsplit * s.q_all;
    case kKComb: return s.fp64 ? 0 : cdiv(s.ntiles, 4);
    case kKP64: return s.fp64 ? cdiv((int64_t)s.m * (s.m - 1) / 2, 4) : 0;
    case kKRowk: return cdiv(s.m, 4);
    case kKSel: return 1;
    case kKRes: return s.m > 2 ? s.m - 1 : 0;
    case kKFeat: return s.feat ? cdiv(s.m, 4) : 0;
    case kKMlp: return s.learned ? cdiv(s.m, 16) : 0;
    case kKTopk: return s.learned ? 1 : 0;
    case kKPairC: return s.learned ? s.nct * 2 * s.nsplit_c * s.q_rows : 0;
    case kKCombC: return s.learned ? cdiv(s.nct, 4) : 0;
    case kKRowkC: return s.learned ? cdiv(s.k, 4) : 0;
    case kKColC: return s.learned ? cdiv(s.m, 64) : 0;
    case kKLsel: return s.learned ? 1 : 0;
    case kKWit: return s.learned ? s.m : 0;
    case kKPairE: return s.nct3 * 2 * s.nsplit * s.q_rows;
    case kKBoundE: return s.nct3 > 0 ? cdiv(s.nsus, 4) : 0;
    case kKCompE: return s.nct3 > 0 ? 1 : 0;
    case kKPairS: return s.nct2 * 2 * s.nsplit_s * s.q_rows;
    case kKCombS: return cdiv(s.nct2, 4);
    case kKRowkS: return cdiv(s.nsus, 4);
    case kKLsel2: return s.nsus > 0 ? 1 : 0;
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

// K > 0 adds the regions of the learned form.
Layout make_layout(int64_t n, int64_t d, int num_cu, int K = 0);

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
hipError_t launch_gate_schedule(const JobDev* jobs, int njobs, SchedDev sc, hipStream_t st);
// loop: grid smaller than the schedule (gated launches), workgroups walk items
hipError_t launch_pair(const JobDev* jobs, int njobs, SchedDev sc, int grid, int waves,
                       hipStream_t st, bool loop = false);
hipError_t launch_combine(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st);
hipError_t launch_pair64(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st);
hipError_t launch_rowk(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st);
hipError_t launch_select(const JobDev* jobs, int njobs, int t, SchedDev sc, int grid,
                         hipStream_t st);
hipError_t launch_resid(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st);
hipError_t launch_gather_status(const JobDev* jobs, int njobs, int32_t* dst, hipStream_t st);
// FP64 decision of the steps whose choice was deferred as a near-tie (step t).
hipError_t launch_tie(const JobDev* jobs, int njobs, SchedDev sc, int t, int num_cu,
                      hipStream_t st);
// Writes `count` (at most kJobsPerLaunch) job-table entries from kernel arguments.
constexpr int kJobsPerLaunch = 8;
hipError_t launch_set_jobs(JobDev* table, int first, const JobDev* host_jobs, int count,
                           hipStream_t st);

// Learned form (lingam_learned.hip).
hipError_t launch_prop_prep(const float* in, PropDev* out, const JobDev* jobs, int njobs,
                            hipStream_t st);
// The learned pass of step t in three launches: features, scores, top-K; the
// candidate pair kernel; candidate measures and the decision.  `grid` holds
// the host's totals of every kind.
hipError_t launch_learned_front(const JobDev* jobs, int njobs, int t, SchedDev sc,
                                const int32_t* grid, hipStream_t st);
hipError_t launch_pair_cand(const JobDev* jobs, int njobs, SchedDev sc, int grid, int waves,
                            hipStream_t st);
hipError_t launch_learned_back(const JobDev* jobs, int njobs, int t, SchedDev sc,
                               const int32_t* grid, hipStream_t st);
// The second (suspect) pass: its schedule, its pair kernel (a bounded grid that
// walks the items), and combine / row k / exact decision (grid-stride).
hipError_t launch_susp_schedule(const JobDev* jobs, int njobs, SchedDev sc, int stage,
                                int num_cu, Tune tu,
                                hipStream_t st);
hipError_t launch_pair_ext(const JobDev* jobs, int njobs, SchedDev sc, int grid, int waves,
                           hipStream_t st);
hipError_t launch_ext_back(const JobDev* jobs, int njobs, int t, SchedDev sc, int g_bound,
                           int g_comp, hipStream_t st);
hipError_t launch_pair_susp(const JobDev* jobs, int njobs, SchedDev sc, int grid, int waves,
                            hipStream_t st);
hipError_t launch_susp_back(const JobDev* jobs, int njobs, int t, SchedDev sc, int g_comb,
                            int g_rowk, int g_sel, hipStream_t st);

// Training of the network.
constexpr int kTrainParts = 512;  // workgroups of the backward pass (partial gradients)
struct TrainLayout {
  int64_t rows;
  int32_t n_lists;
  int nparts;
  size_t status, prop, score, ds, h1, h2, loss_part, part, total;  // status: int32, 0 = ok
};
TrainLayout make_train_layout(int64_t rows, int32_t n_lists);
// Scores of `rows` feature rows; ws holds a PropDev.
hipError_t launch_scores(const float* prop, const float* feat, int64_t rows, float* score,
                         char* ws, hipStream_t st);
// targets (hard) or weights (soft target distributions; targets then unused).
hipError_t launch_grad(const TrainLayout& T, const float* prop, const float* feat,
                       const int64_t* offsets, const int64_t* targets, const float* weights,
                       float* grad, float* loss, float* score_out, char* ws, hipStream_t st);
hipError_t launch_adam(float* prop, const float* grad, float* m1, float* m2, float lr,
                       float beta1, float beta2, float eps, float c1, float c2, hipStream_t st);

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
  size_t linv;   // double [p * p] inverse of the Cholesky factor
  size_t tmp;    // double [p * d] half-solved right-hand sides
  size_t rho0;   // double [d * d] residual correlations before the ordering
  size_t scr;    // double [d * d] permuted residual covariance, then its Cholesky factor
  size_t y;      // double [d * d] columns of the inverse factor (B0 recurrence)
  size_t tol;    // double         pivot tolerance of the current factorisation
  size_t total;
};

VarLayout make_var_layout(int64_t T, int64_t d, int lags, int num_cu);
// `ws` is the VAR block, `job` the base of the ordering job's regions.
hipError_t launch_var_fit(const VarLayout& V, char* ws, char* job, const float* X, int64_t ldx,
                          float* resid_out, double* M_out, hipStream_t st);
hipError_t launch_save_rho(const VarLayout& V, char* ws, char* job, hipStream_t st);
hipError_t launch_b0(const VarLayout& V, char* ws, char* job, const int32_t* order, double* B0,
                     hipStream_t st);

// Least-squares adjacency from a causal order: one region set per call.
struct AdjLayout {
  int64_t n, d, ldx;  // ldx = n rounded up to 64
  size_t ctrl;   // Ctrl (status only)
  size_t mark;   // int32  [d]   permutation check
  size_t tol;    // double       pivot tolerance
  size_t mu;     // double [d]   column means
  size_t xd;     // double [(d + 1) * ldx] the data, variable-major
  size_t s;      // double [d * d] permuted covariance, then its Cholesky factor
  size_t y;      // double [d * d] columns of the inverse factor
  size_t total;
};

AdjLayout make_adj_layout(int64_t n, int64_t d);
// Zero the status; status kInvalid unless `order` is a permutation and every
// rows[s] (s < n, if rows is given) lies in [0, n_rows).
hipError_t launch_adj_check(const AdjLayout& A, char* ws, const int32_t* order,
                            const int32_t* rows, int64_t n_rows, hipStream_t st);
// B (d x d, row-major) after a passed check; sample s is row s of X, or row
// rows[s]; status kDegenerate on non-finite data or a covariance that is not
// positive definite.
hipError_t launch_adjacency(const AdjLayout& A, char* ws, const float* X, int64_t ldx,
                            const int32_t* rows, const int32_t* order, double* B,
                            hipStream_t st);
// One resample's bootstrap counts (see lingam_bootstrap_accumulate).
hipError_t launch_boot_accumulate(const int32_t* order, const double* B, int d, double thr,
                                  int32_t* order_count, int32_t* edge_count, double* coef_sum,
                                  hipStream_t st);
// The counts divided by the number of resamples (see lingam_bootstrap_finalize).
hipError_t launch_boot_finalize(const int32_t* order_count, const int32_t* edge_count,
                                const double* coef_sum, int d, int32_t n_resamples,
                                double* order_prob, double* edge_prob, double* coef_mean,
                                hipStream_t st);

// Dense FP64 pieces shared by the adjacency and VarLiNGAM.
// In-place Cholesky of the leading p x p block of A (lower triangle holds L;
// the upper triangle and columns >= p are left alone).  Status kDegenerate
// for a pivot <= 1e-13 max |A_jj| or a non-finite one.
hipError_t launch_cholesky(double* A, int64_t lda, int p, double* tol, Ctrl* ctrl,
                           hipStream_t st);
// X (ld ldx) = L^-1 for the lower-triangular p x p L (the upper triangle of
// X's diagonal blocks is written as zero; blocks above them are not touched).
hipError_t launch_tri_inverse(const double* L, int64_t ldl, int p, double* X, int64_t ldx,
                              hipStream_t st);
// C = op(A) B, A lower-triangular M x M (op: A, or A^T when trans), B M x N;
// C must not alias B.
hipError_t launch_trmm(int M, int N, const double* A, int64_t lda, bool trans, const double* B,
                       int64_t ldb, double* C, int64_t ldc, hipStream_t st);
// B (p x p, ld p) = least-squares coefficients of every variable on its order
// predecessors from the Cholesky factor L of the order-permuted covariance;
// B[order[i]][order[k]] for k < i, zero elsewhere.  Y: p x p scratch (L^-1).
hipError_t launch_tri_adjacency(const double* L, int64_t ldl, int p, const int32_t* order,
                                double* B, double* Y, hipStream_t st);
// S[a][b] = sig[o_a] sig[o_b] rho[o_a][o_b].
hipError_t launch_perm_scale(const double* rho, int64_t ldr, const double* sig,
                             const int32_t* order, int d, double* S, hipStream_t st);
// mu = row means of Xd[0..d-1][0..n-1]; S = centred Gram permuted into `order`.
hipError_t launch_cov_perm(const double* Xd, int64_t ldx, int n, int d, const int32_t* order,
                           double* mu, double* S, hipStream_t st);
// theta[t] = (I - B0) M[t], t < lags (d x d each, row-major).
hipError_t launch_lagged_effects(const double* M, const double* B0, int d, int lags,
                                 double* theta, hipStream_t st);

#define LG_HIP(call)                    \
  do {                                  \
    const hipError_t lg_e_ = (call);    \
    if (lg_e_ != hipSuccess) return lg_e_; \
  } while (0)

// Standalone residualisation on a row-major matrix.
size_t resid_ws_size(int64_t n, int64_t d);
hipError_t launch_residualize_rowmajor(float* X, int64_t n, int64_t d, int64_t ldx,
                                       const int32_t* active, int32_t n_active, int32_t exo,
                                       char* ws, hipStream_t st);

}  // namespace lg

// Device helpers shared by the gfx950 kernel sources of the library (not
// installed; each source gets its own copies in an unnamed namespace).
#pragma once

#include "lingam_internal.h"

#include <math.h>

namespace lg {
namespace {

// Constants of the maximum-entropy approximation of differential entropy.
constexpr double kK1 = 79.047;
constexpr double kK2 = 7.4129;
constexpr double kGamma = 0.37457;
constexpr double kHnu = 1.41893853320467274178;  // (1 + ln(2 pi)) / 2
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kLog2e = 1.44269504088896340736;
constexpr double kCollinear = 1e-12;  // |rho| >= 1 - kCollinear is degenerate
constexpr int kLogBlock = 32;         // samples per lane folded into one log2 (product <= 2^32)
constexpr float kS1Start = 9.0f;      // start value (negated) of each lane's log cosh sum

constexpr int32_t kStInvalid = -1;
constexpr int32_t kStDegenerate = -2;

template <typename T>
__host__ __device__ inline T* at(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

__device__ inline void set_status(Ctrl* c, int32_t s) { atomicCAS(&c->status, 0, s); }

__device__ inline double entropy_from_moments(double e_lc, double e_g) {
  const double a = e_lc - kGamma;
  return kHnu - kK1 * a * a - kK2 * e_g * e_g;
}

// One evaluation (one residual direction at one sample).  See the header.
__device__ __forceinline__ void eval_dir(float x, float y, float r, float c1h, float c1l,
                                         float& P, float& S1, float& S2) {
  const float kM2 = (float)(-1.0 / (8.0 * kLog2e));  // rounds with relative error 2.7e-9
  const float t = fmaf(-r, y, x);
  const float at = fabsf(t);
  const float m1 = fmaf(c1h, at, c1l * at);
  const float e1 = __builtin_amdgcn_exp2f(m1);
  P = fmaf(P, e1, P);
  S1 = fmaf(m1, -0.5f, S1);
  const float m2 = (kM2 * m1) * m1;
  const float e2 = __builtin_amdgcn_exp2f(m2);
  S2 = fmaf(t, e2, S2);
}

// One evaluation with the pair's scale constant c1 held per lane (pair_item
// dithers it between its two FP32 neighbours so that its mean over the 64
// lanes is the FP64 value): one multiply instead of the hi + lo product.
__device__ __forceinline__ void eval_dir_lane(float x, float y, float r, float c1, float& P,
                                              float& S1, float& S2) {
  const float kM2 = (float)(-1.0 / (8.0 * kLog2e));  // rounds with relative error 2.7e-9
  const float t = fmaf(-r, y, x);
  const float m1 = c1 * fabsf(t);
  const float e1 = __builtin_amdgcn_exp2f(m1);
  P = fmaf(P, e1, P);
  S1 = fmaf(m1, -0.5f, S1);
  const float m2 = (kM2 * m1) * m1;
  const float e2 = __builtin_amdgcn_exp2f(m2);
  S2 = fmaf(t, e2, S2);
}

// The two FP32 values around c (equal when c is a float) and how many of the
// 64 lanes take the upper one so that the lanes' mean is c to 1/128 of a
// float spacing.
__device__ inline void dither_float(double c, float& lo, float& hi, int& n_hi) {
  const float f = (float)c;
  if ((double)f == c) {
    lo = hi = f;
    n_hi = 0;
    return;
  }
  const float g = (double)f < c ? nextafterf(f, INFINITY) : nextafterf(f, -INFINITY);
  lo = fminf(f, g);
  hi = fmaxf(f, g);
  // hi - lo is a power of two: scale by its exponent instead of dividing
  const double gap = (double)hi - (double)lo;
  n_hi = (int)rint(ldexp(c - (double)lo, 6 - ilogb(gap)));
}

// e^x in FP64 for x <= 0, the exponentials of the FP64 paths (their arguments
// are -2|u| and -u^2/2).  Cody and Waite's reduction x = k ln2 + r, |r| <=
// ln2 / 2, with ln2 split into a 32-bit head (so k * head is exact for |k| <
// 2^21) and the rest; e^r from its Taylor series to degree 12 (the remainder
// is below 2.5e-16 of e^r); 2^k applied exactly by ldexp, which takes results
// below the normal range through the subnormals to 0.  No range checks: the
// arguments are never positive, infinite or NaN.
__host__ __device__ inline double exp_nonpos(double x) {
  constexpr double kLn2Head = 0x1.62e42ffp-1;            // ln 2 to 32 bits
  constexpr double kLn2Rest = -0x1.718432a1b0e26p-35;    // ln 2 - kLn2Head
  const double k = rint(x * kLog2e);
  const double r = fma(-k, kLn2Rest, fma(-k, kLn2Head, x));
  double p = 1.0 / 479001600.0;  // 1/12!
  p = fma(p, r, 1.0 / 39916800.0);
  p = fma(p, r, 1.0 / 3628800.0);
  p = fma(p, r, 1.0 / 362880.0);
  p = fma(p, r, 1.0 / 40320.0);
  p = fma(p, r, 1.0 / 5040.0);
  p = fma(p, r, 1.0 / 720.0);
  p = fma(p, r, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  return ldexp(p, (int)k);
}

// FP64 log cosh and Gaussian-weighted term (marginals and the FP64 pair path).
__device__ inline double logcosh64(double u) {
  const double a = fabs(u);
  return a + log1p(exp(-2.0 * a)) - kLn2;
}
__device__ inline double gauss64(double u) { return u * exp(-0.5 * u * u); }

// R(pi, pj) of two active positions entirely in FP64 from the FP64 residuals
// (the small-m path and the FP64 decision of near-ties): one wave, lanes over
// samples, both residual directions; the result is valid in every lane.
// log cosh u = |u| + log(1 + e^{-2|u|}) - ln 2; the logs of a lane's samples
// are taken as the log of their product (each factor is in (1, 2], so 512 of
// them stay below 2^512), one FP64 log per 512 samples.
__device__ inline double pair_measure64(const JobDev& J, int pi, int pj, int lane) {
  const int si = J.act[pi], sj = J.act[pj];
  double r = J.rho[(int64_t)si * J.d + sj];
  const double lim = 1.0 - kCollinear;
  r = r > lim ? lim : (r < -lim ? -lim : r);
  const double al = 1.0 / sqrt(1.0 - r * r);
  const double* zi = J.zd + (int64_t)si * J.ldz;
  const double* zj = J.zd + (int64_t)sj * J.ldz;
  double a1 = 0.0, a2 = 0.0, b1 = 0.0, b2 = 0.0;
  double pa = 1.0, pb = 1.0;
  int cnt = 0, tot = 0;
  for (int s = lane; s < J.n; s += 64) {
    const double xi = zi[s], xj = zj[s];
    const double u = al * (xi - r * xj), w = al * (xj - r * xi);
    const double au = fabs(u), aw = fabs(w);
    a1 += au;
    b1 += aw;
    pa *= 1.0 + exp_nonpos(-2.0 * au);
    pb *= 1.0 + exp_nonpos(-2.0 * aw);
    a2 += u * exp_nonpos(-0.5 * u * u);
    b2 += w * exp_nonpos(-0.5 * w * w);
    ++tot;
    if (++cnt == 512) {
      a1 += log(pa);
      b1 += log(pb);
      pa = pb = 1.0;
      cnt = 0;
    }
  }
  a1 += log(pa) - (double)tot * kLn2;
  b1 += log(pb) - (double)tot * kLn2;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a1 += __shfl_xor(a1, off);
    a2 += __shfl_xor(a2, off);
    b1 += __shfl_xor(b1, off);
    b2 += __shfl_xor(b2, off);
  }
  const double inv_n = 1.0 / (double)J.n;
  const double h_ij = entropy_from_moments(a1 * inv_n, a2 * inv_n);
  const double h_ji = entropy_from_moments(b1 * inv_n, b2 * inv_n);
  return (J.hm[sj] + h_ij) - (J.hm[si] + h_ji);
}

// Pointers read from the job table are generic; the hot loop casts row bases
// to the global address space so loads use global_load with a scalar base.
typedef __attribute__((address_space(1))) const char gchar_t;
typedef __attribute__((address_space(1))) const float gfloat_t;

__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Block-wide deterministic FP64 sum (256 threads), result valid in all threads.
__device__ double block_sum_256(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) sh[tid] += sh[tid + off];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Per-thread sums of the five moments kept for every variable: log cosh z,
// z exp(-z^2/2), z^3, z^4, |z|.  log cosh z = |z| + log(1 + e^{-2|z|}) - ln 2;
// the logs are taken as the log of a running product (each factor in (1, 2],
// flushed every 512 samples), one FP64 log per 512 samples.
struct MomAcc {
  double abs_sum = 0.0, log_sum = 0.0, g = 0.0, z3 = 0.0, z4 = 0.0, prod = 1.0;
  int cnt = 0, tot = 0;
  __device__ inline void add(double z) {
    const double a = fabs(z), z2 = z * z;
    abs_sum += a;
    prod *= 1.0 + exp_nonpos(-2.0 * a);
    g += z * exp_nonpos(-0.5 * z2);
    z3 += z2 * z;
    z4 += z2 * z2;
    ++tot;
    if (++cnt == 512) {
      log_sum += log(prod);
      prod = 1.0;
      cnt = 0;
    }
  }
  // the five sums in the order of store_moments
  __device__ inline void sums(double (&acc)[5]) const {
    acc[0] = abs_sum + (log_sum + log(prod)) - (double)tot * kLn2;
    acc[1] = g;
    acc[2] = z3;
    acc[3] = z4;
    acc[4] = abs_sum;
  }
};

// Block-wide deterministic sum of five FP64 values (256 threads): wave
// butterflies, then the four wave totals in order.  `sh` holds 20 doubles.
// The result is valid in thread 0.
__device__ inline void block_sum_5(double (&v)[5], double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 5; ++k)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v[k] += __shfl_xor(v[k], off);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < 5; ++k) sh[k * 4 + wave] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] = ((sh[k * 4] + sh[k * 4 + 1]) + sh[k * 4 + 2]) + sh[k * 4 + 3];
}

// Means of the five moments of variable `slot` and its marginal entropy.
__device__ inline void store_moments(const JobDev& J, int slot, const double (&acc)[5], int n) {
  const double inv = 1.0 / (double)n;
  double* mo = J.mom + (int64_t)slot * 8;
#pragma unroll
  for (int k = 0; k < 5; ++k) mo[k] = acc[k] * inv;
  J.hm[slot] = entropy_from_moments(acc[0] * inv, acc[1] * inv);
}

// Row-major upper-triangular tile index -> (bi, bj), bi <= bj < nb.
__device__ inline void decode_tile(int tile, int nb, int& bi, int& bj) {
  const double B = 2.0 * nb + 1.0;
  int r = (int)((B - sqrt(B * B - 8.0 * (double)tile)) * 0.5);
  r = r < 0 ? 0 : (r > nb - 1 ? nb - 1 : r);
  auto off = [nb](int q) { return q * nb - (q * (q - 1)) / 2; };
  while (r > 0 && off(r) > tile) --r;
  while (r + 1 < nb && off(r + 1) <= tile) ++r;
  bi = r;
  bj = r + (tile - off(r));
}

// ---------------------------------------------------------------------------
// job lookup and schedules
// ---------------------------------------------------------------------------

// Largest j with pre[j] <= b (pre: exclusive prefix sums, pre[njobs] = total);
// that job owns workgroup b and has a non-zero count.
__device__ inline int find_job(const int32_t* __restrict__ pre, int njobs, int b) {
  int lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Workgroup b belongs to job j at local index b - pre[j]; false when b lies
// beyond the schedule (a grid larger than the device's own totals): the
// workgroup then has nothing to do.
__device__ inline bool locate(const int32_t* __restrict__ pre, int njobs, int b, int& j,
                              int& local) {
  j = find_job(pre, njobs, b);
  local = b - pre[j];
  return local < pre[j + 1] - pre[j];
}

// out[0..njobs] = exclusive prefix sums of count(j); one block of 1024 threads.
template <typename F>
__device__ void block_scan(int njobs, F count, int32_t* out, int32_t* sh) {
  const int tid = threadIdx.x;
  const int per = (njobs + 1023) / 1024;
  const int j0 = tid * per, j1 = min(j0 + per, njobs);
  int32_t s = 0;
  for (int j = j0; j < j1; ++j) s += count(j);
  sh[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t v = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += v;
    __syncthreads();
  }
  int32_t run = tid > 0 ? sh[tid - 1] : 0;
  for (int j = j0; j < j1; ++j) {
    out[j] = run;
    run += count(j);
  }
  if (tid == 1023) out[njobs] = sh[1023];
  __syncthreads();
}

struct Best {
  double v;   // measure (NaN mapped to -inf)
  int slot;   // original id
  int pos;    // position in the active list
  double v2;  // runner-up measure
};

__device__ inline bool better(double va, int sa, double vb, int sb) {
  return va > vb || (va == vb && sa < sb);
}

__device__ inline Best merge(const Best& a, const Best& b) {
  Best r;
  if (better(a.v, a.slot, b.v, b.slot)) {
    r = a;
    r.v2 = fmax(a.v2, b.v);
  } else {
    r = b;
    r.v2 = fmax(b.v2, a.v);
  }
  return r;
}

// Grid-stride walk over the workgroup items of a schedule: f(job, local
// index) for items blockIdx.x, blockIdx.x + gridDim.x, ...  (uniform over
// the workgroup, so f may use barriers).
template <typename F>
__device__ __forceinline__ void for_blocks(const int32_t* __restrict__ pre, int njobs, F f) {
  const int total = pre[njobs];
  for (int b = blockIdx.x; b < total; b += gridDim.x) {
    int jb, lb;
    if (!locate(pre, njobs, b, jb, lb)) break;
    f(jb, lb);
  }
}

// Pair moments (the hot loop), shared by the all-pairs kernel and the
// candidate-row kernel of the learned form.  Grid: per job ntiles * 2 * nsplit
// workgroups of 4 waves (all pairs: upper-triangular 8 x 8 tiles of positions;
// candidate rows: (K / 8) x nblk tiles whose i side lists candidates).  A
// workgroup owns an 8 x 8 block of (i, j) variables, one residual direction
// and one range of samples; wave (wi, wj) owns the 4 x 4 sub-block (i in block
// bi, j in block bj).  Lanes stride over samples (coalesced 256 B loads per
// variable row) and every lane keeps 48 running values (16 pairs x {P, S1, S2})
// for its direction.  The wave ends with an FP64 reduction after which lane
// L < 32 holds the total of sum L, stored at
// part[((split * ntiles + tile) * 4 + wave) * 64 + pair * 4 + dir * 2 + which],
// which 0 = S1 (log cosh, offset as described in the header), 1 = S2;
// dir 0 = residual of i on j, dir 1 = of j on i.
// Work items of the pair kernels.  With kLoop false the grid is the schedule
// and workgroup p (after the XCD remap) takes item p.  With kLoop true (gated
// launches whose size the host only bounds) a smaller grid walks the items:
// workgroup p takes items p * chunk .. p * chunk + chunk - 1, chunk =
// ceil(total / G), so a gated-off step costs a few thousand empty workgroups
// instead of the bound.
// Extension mode: the suspect rows against the extension columns only
// (ceil(nsus / 8) x ceil(ne / 8) tiles whose j side lists positions too).
enum PairMode : int { kModeAll = 0, kModeCand = 1, kModeSusp = 2, kModeExt = 3 };

template <int kMode, int W>
__device__ __forceinline__ void pair_item(const JobDev& J, const JobStep& S, int local,
                                          int wave, int lane);

// W waves per workgroup (1, 2 or 4): every (tile, direction, split) item is
// cut into 4 / W consecutive workgroup items, and the wave's quadrant of the
// tile is (workgroup item mod 4 / W) * W + its wave in the workgroup.
template <int kMode, bool kLoop, int W>
__device__ __forceinline__ void pair_tiles(const JobDev* __restrict__ jobs, int njobs,
                                           const JobStep* __restrict__ js,
                                           const int32_t* __restrict__ pre, int G) {
  static_assert(W == 1 || W == 2 || W == 4, "1, 2 or 4 waves per workgroup");
  constexpr int kQ = 4 / W;
  const int lane = threadIdx.x & 63;
  const int lw = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // Workgroups are dispatched round-robin over the 8 XCDs; give every XCD a
  // contiguous range of (job, tile, direction, split) work so that the rows a
  // tile reads are shared in that XCD's L2.
  const int b = blockIdx.x;
  const int Q = G >> 3, R = G & 7, x = b & 7, idx = b >> 3;
  const int p = x * Q + (x < R ? x : R) + idx;
  auto run = [&](int jb, int local) {
    const int item = local / kQ;
    pair_item<kMode, W>(jobs[jb], js[jb], item, (local - item * kQ) * W + lw, lane);
  };
  int jb, local;
  if (!kLoop) {  // the grid is the schedule: one item per workgroup
    if (locate(pre, njobs, p, jb, local)) run(jb, local);
    return;
  }
  const int total = pre[njobs];
  const int chunk = (total + G - 1) / G;
  for (int it = 0; it < chunk; ++it) {
    const int w = p * chunk + it;
    if (w >= total || !locate(pre, njobs, w, jb, local)) break;
    run(jb, local);
  }
}

template <int kMode, int W>
__device__ __forceinline__ void pair_item(const JobDev& J, const JobStep& S, int local,
                                          int wave, int lane) {
  constexpr bool kCand = kMode != kModeAll;
  const int m = S.m;
  // sample split: the full step's for all pairs and the extension columns
  const int nsplit = kMode == kModeCand ? S.nsplit_c
                     : kMode == kModeSusp ? S.nsplit_s
                                          : S.nsplit;
  const int ntiles = kMode == kModeAll    ? S.ntiles
                     : kMode == kModeCand ? S.nct
                     : kMode == kModeSusp ? S.nct2
                                          : S.nct3;
  const int split_len = kMode == kModeCand ? S.split_len_c
                        : kMode == kModeSusp ? S.split_len_s
                                             : S.split_len;
  const int per_tile = 2 * nsplit;
  const int tile = local / per_tile, rem = local - tile * per_tile;
  const int dir = rem / nsplit, split = rem - dir * nsplit;
  int bi, bj;
  if (kCand) {
    const int ncol = kMode == kModeExt ? cdiv(S.ne, kTileVars) : S.nblk;
    bi = tile / ncol;
    bj = tile - bi * ncol;
  } else {
    decode_tile_st(tile, S.nblk, bi, bj);
  }
  const int wi = wave >> 1, wj = wave & 1;
  if (!kCand && bi == bj && wi > wj) return;  // mirror image of quadrant (wj, wi)
  // A quadrant on the diagonal has the same variables on both sides, so its
  // direction-0 walk (a, c) with a != c already holds both residual
  // directions of each of its 6 pairs (a > c: the larger position regressed
  // on the smaller, which is direction 1 of pair (c, a)); its direction-1
  // item has nothing left to do.  Same rows, coefficients and samples per
  // lane as that item would use, so the sums are the same bits.
  const bool diagq = !kCand && bi == bj && wi == wj;
  if (diagq && dir == 1) return;
  // i side: positions bi * 8 + .. (all pairs) or list entries (candidate /
  // suspect rows; list padding holds position m)
  const int i0 = bi * kTileVars + wi * kWaveVars, pj0 = bj * kTileVars + wj * kWaveVars;
  const int32_t* act = J.act;
  const int32_t* list = kMode == kModeCand ? J.cand : J.cand2;
  const int64_t ldz = J.ldz, ldr = J.d;
  auto ipos = [&](int a) { return kCand ? list[i0 + a] : i0 + a; };
  auto jpos = [&](int a) { return kMode == kModeExt ? J.ext[pj0 + a] : pj0 + a; };

  // The wave walks its 4 x 4 block as (a, c): dir 0 scores residual i|j with
  // i = pi0 + a, j = pj0 + c; dir 1 scores residual j|i with j = pj0 + a,
  // i = pi0 + c.  Lane q < 16 computes the coefficients of walk index q.
  // The scale c1 = -2 log2(e) / sqrt(1 - r^2) of a pair is not rounded to one
  // FP32 value (that would scale every sample of the pair by the same
  // rounding error and bias its log cosh moment): lanes below n_hi take the
  // FP32 value above c1, the others the one below, so the lanes' mean is c1
  // to 1/128 of a float spacing and the sample-to-lane assignment carries no
  // bias (a lane's samples are s = lane, lane + 64, ...).
  float my_r = 0.f, my_lo = 0.f, my_hi = 0.f;
  int my_n = 0;
  {
    const int q = lane & 15, a = q >> 2, c = q & 3;
    const int pi = ipos(dir == 0 ? a : c), pj = jpos(dir == 0 ? c : a);
    const bool valid = pi < m && pj < m && pi != pj;
    if (valid) {
      double r = J.rho[(int64_t)act[pi] * ldr + act[pj]];
      const double lim = 1.0 - kCollinear;
      r = r > lim ? lim : (r < -lim ? -lim : r);
      const double c1 = -2.0 * kLog2e * rsqrt(1.0 - r * r);
      my_r = (float)r;
      dither_float(c1, my_lo, my_hi, my_n);
    }
  }
  float kr[16], kc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    kr[q] = readlane_f(my_r, q);
    const float lo = readlane_f(my_lo, q), hi = readlane_f(my_hi, q);
    const int n_hi = __builtin_amdgcn_readlane(my_n, q);
    kc[q] = lane < n_hi ? hi : lo;
  }
  // Row bases (wave-uniform) and a 32-bit per-lane byte offset, so loads use
  // the scalar-base + vector-offset form.  zr = rows of the regressed
  // variables (the residual's own variable), zx = rows of the regressors.
  gchar_t* zr[4];
  gchar_t* zx[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int pi = ipos(a), pj = jpos(a);
    const int pr = dir == 0 ? pi : pj, px = dir == 0 ? pj : pi;
    // the row ids are wave-uniform: keep them (and the row bases) in SGPRs
    const int sr = __builtin_amdgcn_readfirstlane(pr < m ? act[pr] : J.d);
    const int sx = __builtin_amdgcn_readfirstlane(px < m ? act[px] : J.d);
    zr[a] = (gchar_t*)(J.z + (int64_t)sr * ldz);
    zx[a] = (gchar_t*)(J.z + (int64_t)sx * ldz);
  }

  const int s_begin = split * split_len;
  const int s_end = min(s_begin + split_len, J.n_pad);
  const int nk = (s_end - s_begin) / 64;

  float P[16], S1[16], S2[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    P[q] = 1.f;
    S1[q] = -kS1Start;
    S2[q] = 0.f;
  }
  uint32_t voff = (uint32_t)(s_begin + lane) * 4u;
  float xa[4], xb[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    xa[a] = *(gfloat_t*)(zr[a] + voff);
    xb[a] = *(gfloat_t*)(zx[a] + voff);
  }
  int kb = 0;
  for (int k = 0; k < nk; ++k) {
    // prefetch the next sample of every row; on the last iteration the stride
    // is 0 and the current sample is re-read (always in bounds, no branch)
    const bool more = k + 1 < nk;
    voff += more ? 256u : 0u;
    float na[4], nb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      na[a] = *(gfloat_t*)(zr[a] + voff);
      nb[a] = *(gfloat_t*)(zx[a] + voff);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int q = a * 4 + c;
        eval_dir_lane(xa[a], xb[c], kr[q], kc[q], P[q], S1[q], S2[q]);
      }
    }
    if (++kb == kLogBlock || !more) {
      const float off = 1.5f * (float)kb;  // exact
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        S1[q] += __builtin_amdgcn_logf(P[q]) - off;
        P[q] = 1.f;
      }
      kb = 0;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      xa[a] = na[a];
      xb[a] = nb[a];
    }
  }

  // FP64 sums over the 64 lanes through the wave's own LDS block: lane l
  // writes its 32 sums as column l, then lane L adds, in FP64 and in lane
  // order, sum L & 31 of lanes 32 (L >> 5) .. 32 (L >> 5) + 31, and the two
  // halves are added with one exchange; afterwards lane L < 32 holds sum L.
  // No barrier: a wave's LDS operations complete in the order it issues
  // them, and no other wave touches the block.
  constexpr int kPitch = 68;  // floats per row: 16-byte aligned rows, spread banks
  __shared__ __align__(16) float red[W][32][kPitch];
  float(*T)[kPitch] = red[threadIdx.x >> 6];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    T[2 * q][lane] = S1[q];
    T[2 * q + 1][lane] = S2[q];
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  double v0 = 0.0;
  {
    const float4* row = reinterpret_cast<const float4*>(&T[lane & 31][(lane >> 5) * 32]);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float4 f = row[j];
      v0 += (double)f.x;
      v0 += (double)f.y;
      v0 += (double)f.z;
      v0 += (double)f.w;
    }
  }
  v0 += __shfl_xor(v0, 32);
  if (lane < 32) {
    // sum L = (a * 4 + c) * 2 + which, (a, c) in this direction's walk order;
    // on a diagonal quadrant the walk's lower half is direction 1
    const int a = lane >> 3, c = (lane >> 1) & 3, which = lane & 1;
    const bool flip = dir == 1 || (diagq && a > c);
    const int q = flip ? c * 4 + a : a * 4 + c;  // pair index (i-major) of the tile
    double* part = kMode == kModeAll ? J.part : (kMode == kModeCand ? J.partc : J.parts);
    part[(((int64_t)split * ntiles + tile) * 4 + wave) * 64 + q * 4 + (flip ? 2 : 0) + which] =
        v0;
  }
}

}  // namespace
}  // namespace lg

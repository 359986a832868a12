// gfx950 kernels of the DirectLiNGAM causal-ordering search.
//
// The search (Section 2.2 and Algorithm 1 of AcceleratedLiNGAM) is run with
// the data kept variable-major in the workspace, Z[v][s] (FP32, samples padded
// with zeros to a multiple of 64), and every step is one pass of
//
//   k_pair     pair moments: for every unordered pair {i, j} of active
//              variables, over all samples, the sums that give
//              E[log cosh u] and E[u exp(-u^2/2)] of both standardized
//              regression residuals u = (z_i - rho z_j)/sqrt(1 - rho^2) and
//              u' = (z_j - rho z_i)/sqrt(1 - rho^2).  This is the hot loop.
//   k_combine  maximum-entropy H of both residuals, the likelihood ratio
//              R(i,j) = [H(z_j) + H(u)] - [H(z_i) + H(u')] = -R(j,i)
//   k_rowk     k_i = sum_j min(0, R(i,j))^2
//   k_select   argmax of -k_i (ties -> smallest original id), order[t],
//              swap-remove from the active list
//   k_resid    regress the chosen variable out of every remaining one, keep
//              it standardized, recompute its marginal entropy, and update
//              the correlation matrix by the partial-correlation identity
//
// The correlation matrix is formed once, at the start, by an FP64 MFMA Gram
// (k_gram).  After that the rank-1 least-squares update of the data is
// mirrored exactly on the correlations:
//   rho'_pq = (rho_pq - rho_pe rho_qe) / sqrt((1 - rho_pe^2)(1 - rho_qe^2)),
// which is what a fresh Gram of the updated (standardized) residuals gives in
// exact arithmetic, at O(m^2) instead of O(n m^2) per step.
//
// Arithmetic of the hot loop (per sample, per direction), with u = alpha t,
// t = x - rho y, alpha = 1/sqrt(1 - rho^2):
//   log cosh u = ln2 * ( |u| log2(e) + log2((1 + e^{-2|u|}) / 2) )
//   m1 = -2 alpha log2(e) |t|    (pair constant split hi + lo, one FMA: the
//                                 FP32 rounding of the constant would bias
//                                 every sample the same way)
//   e1 = 2^m1 = e^{-2|u|};  m2 = -m1^2 / (8 log2 e) = -u^2 log2(e) / 2;
//   e2 = 2^m2 = e^{-u^2/2}
//   S1 += -m1/2 ;  P *= (1 + e1) ;  S2 += t e2
// and every kLogBlock samples S1 += log2(P) - 1.5 count, P = 1.  The sum of
// the logs is taken as the log of the product, which leaves two hardware
// transcendentals (v_exp_f32) per evaluation instead of three; subtracting
// 1.5 per sample (exact in FP32) keeps the running sum near its start value
// -kS1Start, so its rounding stays small.  Lane sums are combined in FP64.
//
// Precision: the residuals are kept in FP64 (Zd) and the hot loop reads an
// FP32 copy (Z) rounded afresh at every step; marginal entropies and every
// reduction across lanes, waves and sample splits are FP64.  When few
// variables remain (m <= kFp64MaxM) all pairwise measures are tiny, the step
// is cheap, and k_pair64 computes it entirely in FP64 from Zd.
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
constexpr int kLogBlock = 16;         // samples per lane folded into one log2
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

// FP64 log cosh and Gaussian-weighted term (marginals and the FP64 pair path).
__device__ inline double logcosh64(double u) {
  const double a = fabs(u);
  return a + log1p(exp(-2.0 * a)) - kLn2;
}
__device__ inline double gauss64(double u) { return u * exp(-0.5 * u * u); }

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
// set-up kernels
// ---------------------------------------------------------------------------

__global__ void k_init(int32_t* act, Ctrl* ctrl, int d, int32_t* order) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < d) act[v] = v;
  if (v < (int)(sizeof(Ctrl) / sizeof(int32_t))) reinterpret_cast<int32_t*>(ctrl)[v] = 0;
  if (v == 0 && d == 1) order[0] = 0;
}

// X row-major [n x ldx] -> Zd[v][s] (FP64, exact), zero padding for s >= n and
// for row v == d; row d of the FP32 copy Z is zeroed as well.
__global__ __launch_bounds__(256) void k_ingest(const float* __restrict__ X, int64_t ldx, int n,
                                                int d, int n_pad, double* __restrict__ Zd,
                                                float* __restrict__ Z, int64_t ldz, Ctrl* ctrl) {
  __shared__ float tile[64][65];
  const int s0 = blockIdx.x * 64, v0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  bool bad = false;
  for (int i = 0; i < 16; ++i) {
    const int sl = ty * 16 + i, s = s0 + sl, v = v0 + tx;
    float val = 0.f;
    if (s < n && v < d) {
      val = X[(int64_t)s * ldx + v];
      bad |= !isfinite(val);
    }
    tile[sl][tx] = val;
  }
  __syncthreads();
  for (int i = 0; i < 16; ++i) {
    const int vl = ty * 16 + i, v = v0 + vl, s = s0 + tx;
    if (v <= d && s < n_pad) {
      Zd[(int64_t)v * ldz + s] = (double)tile[tx][vl];
      if (v == d) Z[(int64_t)v * ldz + s] = 0.f;
    }
  }
  if (bad) set_status(ctrl, kStDegenerate);
}

// Population mean and std (two passes, FP64) of each variable.
__global__ __launch_bounds__(256) void k_moments(const double* __restrict__ Zd, int64_t ldz,
                                                 int n, double* mu, double* sig, Ctrl* ctrl) {
  __shared__ double sh[256];
  const int v = blockIdx.x;
  const double* z = Zd + (int64_t)v * ldz;
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += z[k];
  const double m = block_sum_256(s, sh) / (double)n;
  double q = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) {
    const double e = z[k] - m;
    q += e * e;
  }
  const double var = block_sum_256(q, sh) / (double)n;
  if (threadIdx.x == 0) {
    double sd = sqrt(var);
    if (!(sd > 0.0) || !isfinite(sd)) {
      set_status(ctrl, kStDegenerate);
      sd = 1.0;
    }
    mu[v] = m;
    sig[v] = sd;
  }
}

typedef double double4_t __attribute__((ext_vector_type(4)));

// Correlation matrix rho = C / (n sigma_i sigma_j), C = sum_s (x_i - mu_i)(x_j - mu_j),
// on FP64 MFMA (v_mfma_f64_16x16x4f64).  One workgroup per 32 x 32 tile of the
// upper triangle, four waves each owning a 16 x 16 block; samples staged
// through LDS in chunks of 32, centred on the way in.
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ Zd, int64_t ldz,
                                              const double* __restrict__ mu,
                                              const double* __restrict__ sig, int d, int n,
                                              int n_pad, int nb, double* __restrict__ rho,
                                              int64_t ldr, Ctrl* ctrl) {
  constexpr int KC = 32;
  __shared__ double As[KC][33];
  __shared__ double Bs[KC][33];
  int bi, bj;
  decode_tile(blockIdx.x, nb, bi, bj);
  const int I0 = bi * 32, J0 = bj * 32;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  // loader mapping: 32 variables x 32 samples, 4 consecutive samples per thread
  const int lv = tid >> 3, ls = (tid & 7) * 4;
  const int va = I0 + lv, vb = J0 + lv;
  const double* za = Zd + (int64_t)(va < d ? va : d) * ldz;  // row d is all zeros
  const double* zb = Zd + (int64_t)(vb < d ? vb : d) * ldz;
  const double mua = va < d ? mu[va] : 0.0, mub = vb < d ? mu[vb] : 0.0;
  double4_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int s0 = 0; s0 < n_pad; s0 += KC) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int s = s0 + ls + u;
      const bool live = s < n;
      As[ls + u][lv] = (live && va < d) ? za[s] - mua : 0.0;
      Bs[ls + u][lv] = (live && vb < d) ? zb[s] - mub : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const double a = As[kk * 4 + (lane >> 4)][wi * 16 + (lane & 15)];
      const double b = Bs[kk * 4 + (lane >> 4)][wj * 16 + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
  }
  // output layout of the 16x16x4 f64 MFMA: register r of lane l holds
  // D[4 r + l / 16][l % 16]
  bool degenerate = false;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = I0 + wi * 16 + 4 * r + (lane >> 4);
    const int j = J0 + wj * 16 + (lane & 15);
    if (i < d && j < d && (bi != bj || i <= j)) {
      double v = acc[r] / ((double)n * sig[i] * sig[j]);
      if (i == j) v = 1.0;
      else if (!(fabs(v) < 1.0 - kCollinear)) degenerate = true;
      rho[(int64_t)i * ldr + j] = v;
      rho[(int64_t)j * ldr + i] = v;
    }
  }
  if (degenerate) set_status(ctrl, kStDegenerate);
}

// z = (x - mu) / sigma in place in FP64, its FP32 copy, and the marginal
// entropy H(z) of every variable (FP64).
__global__ __launch_bounds__(256) void k_standardize(double* __restrict__ Zd,
                                                     float* __restrict__ Z, int64_t ldz, int n,
                                                     int n_pad, const double* __restrict__ mu,
                                                     const double* __restrict__ sig,
                                                     double* __restrict__ hm) {
  __shared__ double sh[256];
  const int v = blockIdx.x;
  double* zd = Zd + (int64_t)v * ldz;
  float* zf = Z + (int64_t)v * ldz;
  const double m = mu[v], is = 1.0 / sig[v];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < n_pad; k += 256) {
    if (k < n) {
      const double z = (zd[k] - m) * is;
      zd[k] = z;
      zf[k] = (float)z;
      a += logcosh64(z);
      b += gauss64(z);
    } else {
      zf[k] = 0.f;
    }
  }
  const double t1 = block_sum_256(a, sh);
  const double t2 = block_sum_256(b, sh);
  if (threadIdx.x == 0) hm[v] = entropy_from_moments(t1 / n, t2 / n);
}

// ---------------------------------------------------------------------------
// the step kernels
// ---------------------------------------------------------------------------

// Pair moments.  Grid: ntiles * 2 * nsplit workgroups of 4 waves.  A
// workgroup owns an 8 x 8 block of (i, j) positions, one residual direction and
// one range of samples; wave (wi, wj) owns the 4 x 4 sub-block (i in block bi,
// j in block bj).  Lanes stride over samples (coalesced 256 B loads per
// variable row) and every lane keeps 48 running values (16 pairs x {P, S1, S2})
// for its direction.  The wave ends with an FP64 reduction after which lane
// L < 32 holds the total of sum L, stored at
// part[((split * ntiles + tile) * 4 + wave) * 64 + (L / 2) * 4 + dir * 2 + L % 2].
// Sum index (a * 4 + b) * 2 + which, which 0 = S1 (log cosh, offset as described
// in the header), 1 = S2; dir 0 = residual of i on j, dir 1 = of j on i.
__global__ __launch_bounds__(256) void k_pair(const float* __restrict__ Z, int64_t ldz,
                                              const double* __restrict__ rho, int64_t ldr,
                                              const int32_t* __restrict__ act, int m, int nblk,
                                              int ntiles, int nsplit, int split_len, int n_pad,
                                              int zero_slot, double* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // Workgroups are dispatched round-robin over the 8 XCDs; give every XCD a
  // contiguous range of (tile, direction, split) work so that the rows a tile
  // reads are shared in that XCD's L2.
  const int per_tile = 2 * nsplit;
  const int G = ntiles * per_tile;
  const int b = blockIdx.x;
  const int Q = G >> 3, R = G & 7, x = b & 7, idx = b >> 3;
  const int w = x * Q + (x < R ? x : R) + idx;
  const int tile = w / per_tile, rem = w - tile * per_tile;
  const int dir = rem / nsplit, split = rem - dir * nsplit;
  int bi, bj;
  decode_tile(tile, nblk, bi, bj);
  const int wi = wave >> 1, wj = wave & 1;
  if (bi == bj && wi > wj) return;  // mirror image of quadrant (wj, wi)
  const int pi0 = bi * kTileVars + wi * kWaveVars, pj0 = bj * kTileVars + wj * kWaveVars;

  // The wave walks its 4 x 4 block as (a, c): dir 0 scores residual i|j with
  // i = pi0 + a, j = pj0 + c; dir 1 scores residual j|i with j = pj0 + a,
  // i = pi0 + c.  Lane q < 16 computes the coefficients of walk index q.
  float my_r = 0.f, my_c1h = 0.f, my_c1l = 0.f;
  {
    const int q = lane & 15, a = q >> 2, c = q & 3;
    const int pi = pi0 + (dir == 0 ? a : c), pj = pj0 + (dir == 0 ? c : a);
    if (pi < m && pj < m && pi < pj) {
      double r = rho[(int64_t)act[pi] * ldr + act[pj]];
      const double lim = 1.0 - kCollinear;
      r = r > lim ? lim : (r < -lim ? -lim : r);
      const double c1 = -2.0 * kLog2e / sqrt(1.0 - r * r);
      my_r = (float)r;
      my_c1h = (float)c1;
      my_c1l = (float)(c1 - (double)my_c1h);
    }
  }
  float kr[16], kh[16], kl[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    kr[q] = readlane_f(my_r, q);
    kh[q] = readlane_f(my_c1h, q);
    kl[q] = readlane_f(my_c1l, q);
  }
  // Row bases (wave-uniform) and a 32-bit per-lane byte offset, so loads use
  // the scalar-base + vector-offset form.  zr = rows of the regressed
  // variables (the residual's own variable), zx = rows of the regressors.
  const int pr0 = dir == 0 ? pi0 : pj0, px0 = dir == 0 ? pj0 : pi0;
  const char* zr[4];
  const char* zx[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int pr = pr0 + a, px = px0 + a;
    zr[a] = reinterpret_cast<const char*>(Z + (int64_t)(pr < m ? act[pr] : zero_slot) * ldz);
    zx[a] = reinterpret_cast<const char*>(Z + (int64_t)(px < m ? act[px] : zero_slot) * ldz);
  }

  const int s_begin = split * split_len;
  const int s_end = min(s_begin + split_len, n_pad);
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
    xa[a] = *reinterpret_cast<const float*>(zr[a] + voff);
    xb[a] = *reinterpret_cast<const float*>(zx[a] + voff);
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
      na[a] = *reinterpret_cast<const float*>(zr[a] + voff);
      nb[a] = *reinterpret_cast<const float*>(zx[a] + voff);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int q = a * 4 + c;
        eval_dir(xa[a], xb[c], kr[q], kh[q], kl[q], P[q], S1[q], S2[q]);
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

  // FP64 reduction over the 64 lanes: fold the upper half onto the lower, then
  // a reduce-scatter butterfly over 32 lanes; afterwards lane L < 32 holds sum L.
  double v[32];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    v[2 * q] = (double)S1[q];
    v[2 * q + 1] = (double)S2[q];
  }
#pragma unroll
  for (int k2 = 0; k2 < 32; ++k2) v[k2] += __shfl_xor(v[k2], 32);
#pragma unroll
  for (int half = 16; half >= 1; half >>= 1) {
    const bool up = (lane & half) != 0;
#pragma unroll
    for (int k2 = 0; k2 < half; ++k2) {
      const double lo = v[k2], hi = v[k2 + half];
      const double send = up ? lo : hi;
      const double keep = up ? hi : lo;
      v[k2] = keep + __shfl_xor(send, half);
    }
  }
  if (lane < 32) {
    // sum L = (a * 4 + c) * 2 + which, (a, c) in this direction's walk order
    const int a = lane >> 3, c = (lane >> 1) & 3, which = lane & 1;
    const int q = dir == 0 ? a * 4 + c : c * 4 + a;  // pair index (i-major) of the tile
    part[(((int64_t)split * ntiles + tile) * 4 + wave) * 64 + q * 4 + dir * 2 + which] = v[0];
  }
}

// Sum the sample splits (FP64, fixed order), form both residual entropies and
// the likelihood ratio of every pair, write R by position (antisymmetric).
// s1_bias undoes the offsets of the S1 sums: nsplit * 64 * kS1Start + 0.5 n_pad.
__global__ __launch_bounds__(256) void k_combine(const double* __restrict__ part,
                                                 const double* __restrict__ rho, int64_t ldr,
                                                 const int32_t* __restrict__ act,
                                                 const double* __restrict__ hm, int m, int nblk,
                                                 int ntiles, int nsplit, double s1_bias,
                                                 double inv_n, double* __restrict__ rmat,
                                                 int64_t ldm) {
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= ntiles * 64) return;
  const int tile = gid >> 6, wave = (gid >> 4) & 3, q = gid & 15;
  int bi, bj;
  decode_tile(tile, nblk, bi, bj);
  const int wi = wave >> 1, wj = wave & 1;
  const int pi = bi * kTileVars + wi * kWaveVars + (q >> 2);
  const int pj = bj * kTileVars + wj * kWaveVars + (q & 3);
  if (!(pi < m && pj < m && pi < pj)) return;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int sp = 0; sp < nsplit; ++sp) {
    const double* src = part + (((int64_t)sp * ntiles + tile) * 4 + wave) * 64 + q * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] += src[c];
  }
  const int si = act[pi], sj = act[pj];
  double r = rho[(int64_t)si * ldr + sj];
  const double lim = 1.0 - kCollinear;
  r = r > lim ? lim : (r < -lim ? -lim : r);
  const double al = 1.0 / sqrt(1.0 - r * r);
  const double h_ij = entropy_from_moments(kLn2 * (s[0] + s1_bias) * inv_n, al * s[1] * inv_n);
  const double h_ji = entropy_from_moments(kLn2 * (s[2] + s1_bias) * inv_n, al * s[3] * inv_n);
  const double R = (hm[sj] + h_ij) - (hm[si] + h_ji);
  rmat[(int64_t)pi * ldm + pj] = R;
  rmat[(int64_t)pj * ldm + pi] = -R;
}

// The same measure entirely in FP64 from the FP64 residuals, for steps with few
// active variables.  One wave per unordered pair (both directions), lanes over
// samples, FP64 wave reduction; writes R(i,j) and R(j,i) = -R(i,j).
__global__ __launch_bounds__(256) void k_pair64(const double* __restrict__ Zd, int64_t ldz,
                                                const double* __restrict__ rho, int64_t ldr,
                                                const int32_t* __restrict__ act, int m,
                                                const double* __restrict__ hm, int n,
                                                double* __restrict__ rmat, int64_t ldm) {
  const int lane = threadIdx.x & 63;
  const int pair = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int npairs = m * (m - 1) / 2;
  if (pair >= npairs) return;
  int pi = 0, rem = pair;
  while (rem >= m - 1 - pi) {
    rem -= m - 1 - pi;
    ++pi;
  }
  const int pj = pi + 1 + rem;
  const int si = act[pi], sj = act[pj];
  double r = rho[(int64_t)si * ldr + sj];
  const double lim = 1.0 - kCollinear;
  r = r > lim ? lim : (r < -lim ? -lim : r);
  const double al = 1.0 / sqrt(1.0 - r * r);
  const double* zi = Zd + (int64_t)si * ldz;
  const double* zj = Zd + (int64_t)sj * ldz;
  double a1 = 0.0, a2 = 0.0, b1 = 0.0, b2 = 0.0;
  for (int s = lane; s < n; s += 64) {
    const double xi = zi[s], xj = zj[s];
    const double u = al * (xi - r * xj), w = al * (xj - r * xi);
    a1 += logcosh64(u);
    a2 += gauss64(u);
    b1 += logcosh64(w);
    b2 += gauss64(w);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    a1 += __shfl_xor(a1, off);
    a2 += __shfl_xor(a2, off);
    b1 += __shfl_xor(b1, off);
    b2 += __shfl_xor(b2, off);
  }
  if (lane == 0) {
    const double inv_n = 1.0 / (double)n;
    const double h_ij = entropy_from_moments(a1 * inv_n, a2 * inv_n);
    const double h_ji = entropy_from_moments(b1 * inv_n, b2 * inv_n);
    const double R = (hm[sj] + h_ij) - (hm[si] + h_ji);
    rmat[(int64_t)pi * ldm + pj] = R;
    rmat[(int64_t)pj * ldm + pi] = -R;
  }
}

// k_p = sum_{q != p} min(0, R(p, q))^2, one wave per row; mvec[p] = -k_p.
__global__ __launch_bounds__(256) void k_rowk(const double* __restrict__ rmat, int64_t ldm, int m,
                                              double* __restrict__ mvec) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = blockIdx.x * 4 + wave;
  if (p >= m) return;
  const double* row = rmat + (int64_t)p * ldm;
  double k = 0.0;
  for (int q = lane; q < m; q += 64) {
    if (q == p) continue;
    const double x = row[q];
    const double ng = x < 0.0 ? x : 0.0;
    k += ng * ng;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) k += __shfl_xor(k, off);
  if (lane == 0) mvec[p] = -k;
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

// Argmax with tie-break on the original id, teacher forcing, per-step outputs,
// swap-remove of the chosen variable.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_select(const double* __restrict__ mvec,
                                                 int32_t* __restrict__ act, int m, int t, int d,
                                                 Ctrl* ctrl, int32_t* __restrict__ order,
                                                 const int32_t* __restrict__ forced,
                                                 int forced_len, double* step_measures,
                                                 double* step_gap) {
  __shared__ Best sh[1024];
  __shared__ int forced_pos;
  const int tid = threadIdx.x;
  if (tid == 0) forced_pos = -1;
  __syncthreads();
  Best b{-INFINITY, 0x7fffffff, -1, -INFINITY};
  const bool force = t < forced_len;
  const int want = force ? forced[t] : -1;
  for (int p = tid; p < m; p += 1024) {
    double v = mvec[p];
    if (v != v) v = -INFINITY;
    const int sl = act[p];
    Best c{v, sl, p, -INFINITY};
    b = (b.pos < 0) ? c : merge(b, c);
    if (sl == want) forced_pos = p;  // at most one position matches
  }
  sh[tid] = b;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (tid < off) {
      const Best o = sh[tid + off];
      if (o.pos >= 0) sh[tid] = (sh[tid].pos < 0) ? o : merge(sh[tid], o);
    }
    __syncthreads();
  }
  const Best best = sh[0];
  int pos = best.pos;
  if (force) {
    if (forced_pos < 0) {
      if (tid == 0) set_status(ctrl, kStInvalid);
    } else {
      pos = forced_pos;
    }
  }
  if (step_measures) {
    double* row = step_measures + (int64_t)t * d;
    for (int v = tid; v < d; v += 1024) row[v] = NAN;
    __syncthreads();
    for (int p = tid; p < m; p += 1024) row[act[p]] = mvec[p];
  }
  __syncthreads();
  if (tid == 0) {
    const int slot = act[pos];
    order[t] = slot;
    ctrl->exo_slot = slot;
    ctrl->exo_pos = pos;
    if (step_gap) step_gap[t] = best.v - best.v2;
    act[pos] = act[m - 1];
    if (m == 2) order[t + 1] = act[0];
  }
}

// Remove the chosen variable e from every remaining variable p and keep p
// standardized: z_p <- (z_p - rho_pe z_e) / sqrt(1 - rho_pe^2) in FP64, refresh
// the FP32 copy, recompute H(z_p) in FP64, update row p of the correlation
// matrix.  One workgroup per remaining variable.
__global__ __launch_bounds__(256) void k_resid(double* __restrict__ Zd, float* __restrict__ Z,
                                               int64_t ldz, double* __restrict__ rho,
                                               int64_t ldr, const int32_t* __restrict__ act,
                                               int m_after, Ctrl* ctrl,
                                               double* __restrict__ hm, int n, int n_pad) {
  __shared__ double sh[256];
  const int p = blockIdx.x;
  const int sp = act[p], se = ctrl->exo_slot;
  const double* rho_e = rho + (int64_t)se * ldr;
  const double r = rho_e[sp];
  double om = 1.0 - r * r;
  if (!(fabs(r) < 1.0 - kCollinear)) {
    if (threadIdx.x == 0) set_status(ctrl, kStDegenerate);
    om = 1.0;
  }
  const double al = 1.0 / sqrt(om);
  double* zp = Zd + (int64_t)sp * ldz;
  const double* ze = Zd + (int64_t)se * ldz;
  float* zf = Z + (int64_t)sp * ldz;
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < n_pad; k += 256) {
    const double z = al * (zp[k] - r * ze[k]);  // padded samples stay 0
    zp[k] = z;
    zf[k] = (float)z;
    if (k < n) {
      a += logcosh64(z);
      b += gauss64(z);
    }
  }
  const double t1 = block_sum_256(a, sh);
  const double t2 = block_sum_256(b, sh);
  if (threadIdx.x == 0) hm[sp] = entropy_from_moments(t1 / n, t2 / n);
  double* rho_p = rho + (int64_t)sp * ldr;
  for (int q = threadIdx.x; q < m_after; q += 256) {
    if (q == p) continue;
    const int sq = act[q];
    const double rq = rho_e[sq];
    double oq = 1.0 - rq * rq;
    if (!(fabs(rq) < 1.0 - kCollinear)) oq = 1.0;  // flagged by q's own workgroup
    rho_p[sq] = (rho_p[sq] - r * rq) / sqrt(om * oq);
  }
}

__global__ void k_copy_status(const Ctrl* ctrl, int32_t* dst) { dst[0] = ctrl->status; }

// ---------------------------------------------------------------------------
// standalone residualisation on a row-major matrix
// ---------------------------------------------------------------------------

constexpr int kRowsPerBlk = 256;

// partial[blk][c] = sum over rows of the block of f(x_c); c = n_active is exo.
// centred == 0: f = x; centred == 1: f = (x_c - mu_c) (x_e - mu_e).
__global__ __launch_bounds__(256) void k_rr_partial(const float* __restrict__ X, int64_t ldx,
                                                    int n, int d,
                                                    const int32_t* __restrict__ active,
                                                    int n_active, int exo,
                                                    const double* __restrict__ mean,
                                                    int centred, double* __restrict__ partial,
                                                    int32_t* status) {
  const int blk = blockIdx.x;
  const int r0 = blk * kRowsPerBlk, r1 = min(r0 + kRowsPerBlk, n);
  for (int c = threadIdx.x; c <= n_active; c += 256) {
    const int col = c < n_active ? active[c] : exo;
    double s = 0.0;
    if (col < 0 || col >= d) {  // bad id in `active`: report, touch nothing
      atomicCAS(status, 0, kStInvalid);
      partial[(int64_t)blk * (n_active + 1) + c] = 0.0;
      continue;
    }
    if (!centred) {
      for (int r = r0; r < r1; ++r) s += (double)X[(int64_t)r * ldx + col];
    } else {
      const double mc = mean[c], me = mean[n_active];
      for (int r = r0; r < r1; ++r)
        s += ((double)X[(int64_t)r * ldx + col] - mc) * ((double)X[(int64_t)r * ldx + exo] - me);
    }
    partial[(int64_t)blk * (n_active + 1) + c] = s;
  }
}

// out[c] = sum_blk partial[blk][c] / n  (fixed order)
__global__ void k_rr_reduce(const double* __restrict__ partial, int nblk, int n_active, int n,
                            double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > n_active) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * (n_active + 1) + c];
  out[c] = s / (double)n;
}

__global__ __launch_bounds__(256) void k_rr_apply(float* __restrict__ X, int64_t ldx, int n,
                                                  int d, const int32_t* __restrict__ active,
                                                  int n_active, int exo,
                                                  const double* __restrict__ cov,
                                                  int32_t* status) {
  if (status[0] != 0) return;  // an id was out of range: leave X untouched
  const double ve = cov[n_active];
  if (!(ve > 0.0)) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) atomicCAS(status, 0, kStDegenerate);
    return;
  }
  const int c = blockIdx.y;
  const int col = active[c];
  if (col == exo || col < 0 || col >= d) return;
  const double b = cov[c] / ve;
  for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
    const int64_t o = (int64_t)r * ldx;
    X[o + col] = (float)((double)X[o + col] - b * (double)X[o + exo]);
  }
}

__global__ void k_zero_i32(int32_t* p) { p[0] = 0; }

}  // namespace

// ---------------------------------------------------------------------------
// host side: plans, layout, launchers
// ---------------------------------------------------------------------------

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

StepPlan plan_step(int64_t m, int64_t n_pad, int num_cu) {
  StepPlan p;
  p.nblk = (int)((m + kTileVars - 1) / kTileVars);
  p.ntiles = p.nblk * (p.nblk + 1) / 2;
  const int64_t iters = n_pad / kSampleQuantum;
  // Enough workgroups (two per tile, one per residual direction) to fill every
  // CU several times over: when the pair triangle is small, split the sample
  // range (partials are combined in FP64), keeping at least kMinIters sample
  // iterations per split so the per-workgroup set-up and reduction stay small.
  constexpr int64_t kMinIters = 8;
  const int64_t target = (int64_t)num_cu * 16;
  int64_t ns = (target + 2 * p.ntiles - 1) / (2 * p.ntiles);
  const int64_t cap = iters >= kMinIters ? iters / kMinIters : 1;
  if (ns > cap) ns = cap;
  if (ns < 1) ns = 1;
  const int64_t per = (iters + ns - 1) / ns;
  p.split_len = (int)(per * kSampleQuantum);
  p.nsplit = (int)((iters + per - 1) / per);
  return p;
}

Layout make_layout(int64_t n, int64_t d, int num_cu) {
  Layout L{};
  L.n = n;
  L.d = d;
  L.n_pad = (n + kSampleQuantum - 1) / kSampleQuantum * kSampleQuantum;
  L.ldz = L.n_pad;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.zd = take(sizeof(double) * (size_t)(d + 1) * (size_t)L.ldz);
  L.z = take(sizeof(float) * (size_t)(d + 1) * (size_t)L.ldz);
  L.mu = take(sizeof(double) * (size_t)d);
  L.sig = take(sizeof(double) * (size_t)d);
  L.rho = take(sizeof(double) * (size_t)d * (size_t)d);
  L.hm = take(sizeof(double) * (size_t)d);
  L.act = take(sizeof(int32_t) * (size_t)d);
  L.ctrl = take(sizeof(Ctrl));
  size_t pe = 0;
  for (int64_t m = d; m > kFp64MaxM; --m) {
    const StepPlan p = plan_step(m, L.n_pad, num_cu);
    const size_t need = (size_t)p.ntiles * (size_t)p.nsplit * 256;
    if (need > pe) pe = need;
  }
  L.part_elems = pe;
  L.part = take(sizeof(double) * (pe ? pe : 1));
  L.rmat = take(sizeof(double) * (size_t)d * (size_t)d);
  L.mvec = take(sizeof(double) * (size_t)d);
  L.total = off;
  return L;
}

hipError_t launch_init(const Layout& L, char* ws, int32_t* order, hipStream_t st) {
  const int threads = 256;
  const int64_t cnt = L.d > 64 ? L.d : 64;
  hipLaunchKernelGGL(k_init, dim3((unsigned)((cnt + threads - 1) / threads)), dim3(threads), 0,
                     st, at<int32_t>(ws, L.act), at<Ctrl>(ws, L.ctrl), (int)L.d, order);
  return hipGetLastError();
}

hipError_t launch_ingest(const Layout& L, char* ws, const float* X, int64_t ldx,
                         hipStream_t st) {
  dim3 grid((unsigned)(L.n_pad / 64), (unsigned)((L.d + 1 + 63) / 64));
  hipLaunchKernelGGL(k_ingest, grid, dim3(256), 0, st, X, ldx, (int)L.n, (int)L.d,
                     (int)L.n_pad, at<double>(ws, L.zd), at<float>(ws, L.z), L.ldz,
                     at<Ctrl>(ws, L.ctrl));
  return hipGetLastError();
}

hipError_t launch_moments(const Layout& L, char* ws, hipStream_t st) {
  hipLaunchKernelGGL(k_moments, dim3((unsigned)L.d), dim3(256), 0, st, at<double>(ws, L.zd),
                     L.ldz, (int)L.n, at<double>(ws, L.mu), at<double>(ws, L.sig),
                     at<Ctrl>(ws, L.ctrl));
  return hipGetLastError();
}

hipError_t launch_gram(const Layout& L, char* ws, hipStream_t st) {
  const int nb = (int)((L.d + 31) / 32);
  const int tiles = nb * (nb + 1) / 2;
  hipLaunchKernelGGL(k_gram, dim3((unsigned)tiles), dim3(256), 0, st, at<double>(ws, L.zd),
                     L.ldz, at<double>(ws, L.mu), at<double>(ws, L.sig), (int)L.d, (int)L.n,
                     (int)L.n_pad, nb, at<double>(ws, L.rho), L.d, at<Ctrl>(ws, L.ctrl));
  return hipGetLastError();
}

hipError_t launch_standardize(const Layout& L, char* ws, hipStream_t st) {
  hipLaunchKernelGGL(k_standardize, dim3((unsigned)L.d), dim3(256), 0, st,
                     at<double>(ws, L.zd), at<float>(ws, L.z), L.ldz, (int)L.n, (int)L.n_pad,
                     at<double>(ws, L.mu), at<double>(ws, L.sig), at<double>(ws, L.hm));
  return hipGetLastError();
}

hipError_t launch_pair(const Layout& L, char* ws, int m, const StepPlan& p, hipStream_t st) {
  const int G = p.ntiles * 2 * p.nsplit;
  hipLaunchKernelGGL(k_pair, dim3((unsigned)G), dim3(256), 0, st, at<float>(ws, L.z), L.ldz,
                     at<double>(ws, L.rho), L.d, at<int32_t>(ws, L.act), m, p.nblk, p.ntiles,
                     p.nsplit, p.split_len, (int)L.n_pad, (int)L.d, at<double>(ws, L.part));
  return hipGetLastError();
}

hipError_t launch_combine(const Layout& L, char* ws, int m, const StepPlan& p, hipStream_t st) {
  const int64_t threads = (int64_t)p.ntiles * 64;
  const double s1_bias = (double)p.nsplit * 64.0 * (double)kS1Start + 0.5 * (double)L.n_pad;
  hipLaunchKernelGGL(k_combine, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st,
                     at<double>(ws, L.part), at<double>(ws, L.rho), L.d,
                     at<int32_t>(ws, L.act), at<double>(ws, L.hm), m, p.nblk, p.ntiles,
                     p.nsplit, s1_bias, 1.0 / (double)L.n, at<double>(ws, L.rmat), L.d);
  return hipGetLastError();
}

hipError_t launch_pair64(const Layout& L, char* ws, int m, hipStream_t st) {
  const int npairs = m * (m - 1) / 2;
  hipLaunchKernelGGL(k_pair64, dim3((unsigned)((npairs + 3) / 4)), dim3(256), 0, st,
                     at<double>(ws, L.zd), L.ldz, at<double>(ws, L.rho), L.d,
                     at<int32_t>(ws, L.act), m, at<double>(ws, L.hm), (int)L.n,
                     at<double>(ws, L.rmat), L.d);
  return hipGetLastError();
}

hipError_t launch_rowk(const Layout& L, char* ws, int m, hipStream_t st) {
  hipLaunchKernelGGL(k_rowk, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st,
                     at<double>(ws, L.rmat), L.d, m, at<double>(ws, L.mvec));
  return hipGetLastError();
}

hipError_t launch_select(const Layout& L, char* ws, int m, int t, int32_t* order,
                         const int32_t* forced, int forced_len, double* step_measures,
                         double* step_gap, hipStream_t st) {
  hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, st, at<double>(ws, L.mvec),
                     at<int32_t>(ws, L.act), m, t, (int)L.d, at<Ctrl>(ws, L.ctrl), order, forced,
                     forced_len, step_measures, step_gap);
  return hipGetLastError();
}

hipError_t launch_resid(const Layout& L, char* ws, int m_after, hipStream_t st) {
  hipLaunchKernelGGL(k_resid, dim3((unsigned)m_after), dim3(256), 0, st, at<double>(ws, L.zd),
                     at<float>(ws, L.z), L.ldz, at<double>(ws, L.rho), L.d,
                     at<int32_t>(ws, L.act), m_after, at<Ctrl>(ws, L.ctrl),
                     at<double>(ws, L.hm), (int)L.n, (int)L.n_pad);
  return hipGetLastError();
}

hipError_t launch_copy_status(const Layout& L, char* ws, int32_t* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(1), 0, st, at<Ctrl>(ws, L.ctrl), dst);
  return hipGetLastError();
}

// workspace of the standalone residualisation:
// [status int32 (256 B)] [mean double[d+1]] [cov double[d+1]] [partial double[nblk*(d+1)]]
size_t resid_ws_size(int64_t n, int64_t d) {
  const int64_t nblk = (n + kRowsPerBlk - 1) / kRowsPerBlk;
  return 256 + align256(sizeof(double) * (size_t)(d + 1)) * 2 +
         align256(sizeof(double) * (size_t)nblk * (size_t)(d + 1));
}

hipError_t launch_residualize_rowmajor(float* X, int64_t n, int64_t d, int64_t ldx,
                                       const int32_t* active, int32_t n_active, int32_t exo,
                                       char* ws, hipStream_t st) {
  const int64_t nblk = (n + kRowsPerBlk - 1) / kRowsPerBlk;
  int32_t* status = reinterpret_cast<int32_t*>(ws);
  double* mean = reinterpret_cast<double*>(ws + 256);
  double* cov = reinterpret_cast<double*>(ws + 256 + align256(sizeof(double) * (size_t)(d + 1)));
  double* partial =
      reinterpret_cast<double*>(ws + 256 + 2 * align256(sizeof(double) * (size_t)(d + 1)));
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, st, status);
  hipLaunchKernelGGL(k_rr_partial, dim3((unsigned)nblk), dim3(256), 0, st, X, ldx, (int)n,
                     (int)d, active, n_active, exo, (const double*)nullptr, 0, partial, status);
  const unsigned rb = (unsigned)((n_active + 1 + 255) / 256);
  hipLaunchKernelGGL(k_rr_reduce, dim3(rb), dim3(256), 0, st, partial, (int)nblk, n_active,
                     (int)n, mean);
  hipLaunchKernelGGL(k_rr_partial, dim3((unsigned)nblk), dim3(256), 0, st, X, ldx, (int)n,
                     (int)d, active, n_active, exo, mean, 1, partial, status);
  hipLaunchKernelGGL(k_rr_reduce, dim3(rb), dim3(256), 0, st, partial, (int)nblk, n_active,
                     (int)n, cov);
  const int64_t gx = (n + 255) / 256;
  dim3 grid((unsigned)(gx < 64 ? gx : 64), (unsigned)n_active);
  hipLaunchKernelGGL(k_rr_apply, grid, dim3(256), 0, st, X, ldx, (int)n, (int)d, active,
                     n_active, exo, cov, status);
  return hipGetLastError();
}

}  // namespace lg

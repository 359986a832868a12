// gfx950 kernels of the learned-proposal form of the ordering search.
//
// The exact search (Section 2.2, Algorithm 1) spends its time on the measure
// of every pair of active variables.  The learned form evaluates that measure
// only for the rows of K candidates chosen by a small network, and decides on
// the device, without any host round trip, whether the candidates' result can
// stand in for the full step:
//
//   k_features      16 features per active variable (moments of z kept by the
//                   residual update, statistics of its correlation row, rank
//                   of its marginal entropy, progress of the search)
//   k_mlp           scores of a 16 -> 128 -> 128 -> 1 ReLU network, BF16
//                   weights and activations on MFMA, FP32 accumulation
//                   (the same code as the scores entry point's k_scores)
//   k_topk          the K best scores (ties to the smaller original id) by an
//                   8-bit radix select over 64-bit keys (and the extension
//                   columns ranked next, when asked for)
//   k_pair_cand     the pair moments of every (candidate, active) pair: the
//                   all-pairs hot loop on (K / 8) x nblk tiles
//   k_combine_cand  R(c, j) of every candidate row
//   k_cand_k        exact k of every candidate, and for every other variable
//                   l the lower bound sum_c max(0, R(c, l))^2 <= k_l its
//                   candidate pairs give
//   k_pair_wit      for the variables that bound leaves at or below the best
//                   candidate's k: their pair measures against their most
//                   correlated non-candidate variables (witnesses), added to
//                   the bound
//   k_lselect       best candidate; it is certified when every lower bound
//                   exceeds its k; otherwise the suspects (bound <= its k)
//                   are listed for a second pass over their rows, or, when
//                   too many, the best candidate is accepted if its score
//                   beats every non-candidate's by the margin; audit steps
//                   and the rest hand the step to the full kernels (gated by
//                   k_gate_schedule)
//   k_pair_ext, k_ext_bound, k_ext_compact  (optional) the listed suspects
//                   against the extension columns (the variables ranked right
//                   after the candidates), their share added to the bounds,
//                   and the list cut to the suspects still at or below the
//                   best candidate's k (none left: the best candidate is
//                   committed)
//   k_pair_susp, k_combine_susp, k_susp_rowk, k_lselect2  the remaining
//                   suspects' full rows and the exact choice
//
// and the training kernels of the network (forward with saved activations,
// listwise softmax cross-entropy, backward on MFMA, gradient reduction, Adam).
#include "lingam_device.h"

namespace lg {
namespace {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x4_t load4(const uint16_t* p) {
  // 8-byte aligned by construction of every caller's layout
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  bf16x4_t r;
  r[0] = (short)(v.x & 0xFFFF);
  r[1] = (short)(v.x >> 16);
  r[2] = (short)(v.y & 0xFFFF);
  r[3] = (short)(v.y >> 16);
  return r;
}

// 16 x 16 x 16 BF16 MFMA.  Operand layout: lane l supplies A[l % 16][4 (l / 16) + j]
// and B[4 (l / 16) + j][l % 16] (j = 0..3); result register r of lane l is
// D[4 (l / 16) + r][l % 16].
__device__ __forceinline__ f32x4_t mfma16(bf16x4_t a, bf16x4_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

constexpr int kLdW = kHidden + 8;  // padded LDS row of 128 BF16 values
constexpr int kLdR = 64 + 8;       // padded LDS row of 64 BF16 values

// ---------------------------------------------------------------------------
// network preparation
// ---------------------------------------------------------------------------

// FP32 parameter block [mean(16), scale(16), W1, b1, W2, b2, w3, b3] -> BF16
// weights; a non-finite value or a scale <= 0 marks every job invalid (and
// sets *flag when given).
__global__ __launch_bounds__(256) void k_prop_prep(const float* __restrict__ in,
                                                   PropDev* __restrict__ out,
                                                   const JobDev* __restrict__ jobs, int njobs,
                                                   int32_t* __restrict__ flag) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const float* w = in + kPropNorm;
  int mybad = 0;
  for (int i = threadIdx.x; i < kHidden * kHidden; i += 256) {
    const float v = w[kOffW2 + i];
    mybad |= !isfinite(v);
    out->w2[i] = to_bf16(v);
  }
  for (int i = threadIdx.x; i < kHidden * kFeat; i += 256) {
    const float v = w[kOffW1 + i];
    mybad |= !isfinite(v);
    out->w1[i] = to_bf16(v);
  }
  for (int i = threadIdx.x; i < kHidden; i += 256) {
    const float a = w[kOffW3 + i], b1 = w[kOffB1 + i], b2 = w[kOffB2 + i];
    mybad |= !isfinite(a) || !isfinite(b1) || !isfinite(b2);
    out->w3[i] = to_bf16(a);
    out->b1[i] = b1;
    out->b2[i] = b2;
  }
  if (threadIdx.x < kFeat) {
    const float mu = in[threadIdx.x], sd = in[kFeat + threadIdx.x];
    mybad |= !isfinite(mu) || !(sd > 0.f) || !isfinite(sd);
    out->mu[threadIdx.x] = mu;
    out->sd[threadIdx.x] = sd;
  }
  if (threadIdx.x == 0) {
    out->b3 = w[kOffB3];
    mybad |= !isfinite(w[kOffB3]);
  }
  if (mybad) bad = 1;
  __syncthreads();
  if (bad) {
    for (int j = threadIdx.x; j < njobs; j += 256) set_status(jobs[j].ctrl, kStInvalid);
    if (flag && threadIdx.x == 0) *flag = 2;
  }
}

// ---------------------------------------------------------------------------
// features
// ---------------------------------------------------------------------------

// One wave per active position p: statistics of its correlation row and the
// rank of its marginal entropy; lane 0 assembles the 16 features.
__global__ __launch_bounds__(256) void k_features(const JobDev* __restrict__ jobs, int njobs,
                                                  const JobStep* __restrict__ js,
                                                  const int32_t* __restrict__ pre, int t) {
  int jb, lb;
  if (!locate(pre, njobs, blockIdx.x, jb, lb)) return;
  const JobDev& J = jobs[jb];
  const int m = js[jb].m;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lb * 4 + wave;
  if (p >= m) return;
  const int si = J.act[p];
  const double Hi = J.hm[si];
  const double* rr = J.rho + (int64_t)si * J.d;
  double mx = 0.0, s1 = 0.0, s2 = 0.0, sw = 0.0;
  int c5 = 0, rk = 0;
  // this lane's kWit largest |rho| (ties to the smaller position), descending
  double ta[kWit];
  int tq[kWit];
#pragma unroll
  for (int w = 0; w < kWit; ++w) {
    ta[w] = -1.0;
    tq[w] = -1;
  }
  // four positions per lane per pass: their gathers are issued together
  constexpr int kU = 4;
  for (int q0 = lane; q0 < m; q0 += 64 * kU) {
    int sqv[kU];
    double Hv[kU], rv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = q0 + 64 * u;
      sqv[u] = q < m ? J.act[q] : si;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      Hv[u] = J.hm[sqv[u]];
      rv[u] = rr[sqv[u]];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int q = q0 + 64 * u;
      if (q >= m) break;
      const int sq = sqv[u];
      const double Hq = Hv[u];
      rk += (Hq < Hi || (Hq == Hi && sq < si)) ? 1 : 0;  // never true for q == p
      if (q == p) continue;
      const double r = rv[u], a = fabs(r), r2 = r * r;
      mx = fmax(mx, a);
      s1 += a;
      s2 += r2;
      sw += r2 * Hq;
      c5 += a > 0.5 ? 1 : 0;
      // q grows along the lane, so an equal |rho| never displaces an earlier q
      double ca = a;
      int cq = q;
#pragma unroll
      for (int w = 0; w < kWit; ++w) {
        if (ca > ta[w]) {
          const double xa = ta[w];
          const int xq = tq[w];
          ta[w] = ca;
          tq[w] = cq;
          ca = xa;
          cq = xq;
        }
      }
    }
  }
  if (J.wit) {
    // kWit rounds of a wave-wide arg-max over the lanes' list heads
    int head = 0;
    for (int w = 0; w < kWit; ++w) {
      double ba = -1.0;
      int bq = -1;
#pragma unroll
      for (int h = 0; h < kWit; ++h)
        if (h == head) {
          ba = ta[h];
          bq = tq[h];
        }
      double va = ba;
      int vq = bq;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double oa = __shfl_xor(va, off);
        const int oq = __shfl_xor(vq, off);
        if (oa > va || (oa == va && oq >= 0 && (vq < 0 || oq < vq))) {
          va = oa;
          vq = oq;
        }
      }
      if (vq >= 0 && vq == bq && head < kWit) ++head;  // the owner pops its head
      if (lane == 0) J.wit[(int64_t)p * kWit + w] = vq;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off));
    s1 += __shfl_xor(s1, off);
    s2 += __shfl_xor(s2, off);
    sw += __shfl_xor(sw, off);
    c5 += __shfl_xor(c5, off);
    rk += __shfl_xor(rk, off);
  }
  if (lane != 0) return;
  const double* mo = J.mom + (int64_t)si * 8;
  const double mm1 = (double)(m - 1);
  float f[kFeat];
  f[0] = (float)mo[0];
  f[1] = (float)mo[1];
  f[2] = (float)Hi;
  f[3] = (float)mo[2];
  f[4] = (float)(mo[3] - 3.0);
  f[5] = (float)mo[4];
  f[6] = (float)(mo[2] * mo[2]);
  f[7] = (float)mx;
  f[8] = (float)(s2 / (double)m);
  f[9] = (float)(s1 / mm1);
  f[10] = (float)((double)c5 / mm1);
  f[11] = (float)((double)rk / (double)m);
  f[12] = (float)((double)t / (double)J.d);
  f[13] = (float)((double)m / (double)J.d);
  f[14] = (float)log((double)J.n);
  f[15] = (float)(s2 > 0.0 ? sw / s2 : 0.0);
  if (J.feat) {
    float* dst = J.feat + (int64_t)p * kFeat;
#pragma unroll
    for (int k = 0; k < kFeat; ++k) dst[k] = f[k];
  }
  if (J.record) {
    float* rec = J.record + ((int64_t)t * J.d + si) * kFeat;
#pragma unroll
    for (int k = 0; k < kFeat; ++k) rec[k] = f[k];
  }
}

// ---------------------------------------------------------------------------
// the network
// ---------------------------------------------------------------------------

// LDS of one 64-row tile of the network.
struct MlpShared {
  uint16_t w2[kHidden][kLdW];  // W2[h][g]
  uint16_t h1[64][kLdW];       // first hidden layer of the tile's rows (BF16)
};

__device__ inline void stage_w2(const PropDev& W, MlpShared& S) {
  for (int i = threadIdx.x; i < kHidden * kHidden / 4; i += 256) {
    const int h = i / (kHidden / 4), g4 = (i % (kHidden / 4)) * 4;
    *reinterpret_cast<uint2*>(&S.w2[h][g4]) =
        *reinterpret_cast<const uint2*>(&W.w2[h * kHidden + g4]);
  }
}

// Forward pass of rows row0 .. row0 + 63 (rows >= nrows are zero inputs and
// produce nothing).  Wave w owns rows row0 + 16 w .. + 15.  Features are
// normalized with the network's mean and scale and rounded to BF16.  Writes
// score[row]; with H1 / H2 non-NULL also the BF16 first and FP32 second hidden
// layer ([row][128]) for the backward pass.  S.w2 must be staged.
__device__ void mlp_tile(const PropDev& W, MlpShared& S, const float* __restrict__ feat,
                         int64_t row0, int64_t nrows, float* __restrict__ score,
                         uint16_t* __restrict__ H1, float* __restrict__ H2) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg4 = (lane >> 4) * 4;
  // layer 1: A = x[row][f], B = W1^T
  bf16x4_t xa;
  {
    const int64_t row = row0 + wave * 16 + li;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int f = lg4 + j;
      float v = 0.f;
      if (row < nrows) v = (feat[row * kFeat + f] - W.mu[f]) / W.sd[f];
      xa[j] = (short)to_bf16(v);
    }
  }
#pragma unroll
  for (int nt = 0; nt < kHidden / 16; ++nt) {
    const int n = nt * 16 + li;
    const bf16x4_t wb = load4(&W.w1[n * kFeat + lg4]);
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma16(xa, wb, acc);
    const float b = W.b1[n];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float h = fmaxf(acc[r] + b, 0.f);
      S.h1[wave * 16 + lg4 + r][n] = to_bf16(h);
    }
  }
  __syncthreads();
  if (H1) {
    for (int e = lane; e < 16 * kHidden / 4; e += 64) {
      const int i = e / (kHidden / 4), g4 = (e % (kHidden / 4)) * 4;
      const int64_t row = row0 + wave * 16 + i;
      if (row < nrows)
        *reinterpret_cast<uint2*>(&H1[row * kHidden + g4]) =
            *reinterpret_cast<const uint2*>(&S.h1[wave * 16 + i][g4]);
    }
  }
  // layer 2: A = h1[row][g], B = W2^T; score = w3 . relu(.) + b3
  float ps[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
  for (int nt = 0; nt < kHidden / 16; ++nt) {
    const int n = nt * 16 + li;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kHidden / 16; ++ks) {
      const bf16x4_t a = load4(&S.h1[wave * 16 + li][ks * 16 + lg4]);
      const bf16x4_t b = load4(&S.w2[n][ks * 16 + lg4]);
      acc = mfma16(a, b, acc);
    }
    const float b2 = W.b2[n], w3 = from_bf16(W.w3[n]);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float h = fmaxf(acc[r] + b2, 0.f);
      ps[r] = fmaf(h, w3, ps[r]);
      if (H2) {
        const int64_t row = row0 + wave * 16 + lg4 + r;
        if (row < nrows) H2[row * kHidden + n] = h;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) ps[r] += __shfl_xor(ps[r], off);
  if (li == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + wave * 16 + lg4 + r;
      if (row < nrows) score[row] = ps[r] + W.b3;
    }
  }
}

// Inference of rows row0 .. row0 + 15 (rows >= nrows are zero inputs and
// produce nothing): the four waves split the hidden units (wave w owns units
// 32 w .. 32 w + 31 of both layers), share the first layer through LDS and add
// their partial scores in a fixed order.  Same arithmetic as mlp_tile.
struct Mlp16Shared {
  uint16_t h1[16][kLdW];
  float part[4][16];
};

__device__ void mlp16(const PropDev& W, Mlp16Shared& S, const float* __restrict__ feat,
                      int64_t row0, int64_t nrows, float* __restrict__ score) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg4 = (lane >> 4) * 4;
  bf16x4_t xa;
  {
    const int64_t row = row0 + li;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int f = lg4 + j;
      float v = 0.f;
      if (row < nrows) v = (feat[row * kFeat + f] - W.mu[f]) / W.sd[f];
      xa[j] = (short)to_bf16(v);
    }
  }
#pragma unroll
  for (int t2 = 0; t2 < 2; ++t2) {
    const int n = (wave * 2 + t2) * 16 + li;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma16(xa, load4(&W.w1[n * kFeat + lg4]), acc);
    const float b = W.b1[n];
#pragma unroll
    for (int r = 0; r < 4; ++r) S.h1[lg4 + r][n] = to_bf16(fmaxf(acc[r] + b, 0.f));
  }
  __syncthreads();
  float ps[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t2 = 0; t2 < 2; ++t2) {
    const int n = (wave * 2 + t2) * 16 + li;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < kHidden / 16; ++ks)
      acc = mfma16(load4(&S.h1[li][ks * 16 + lg4]),
                   load4(&W.w2[n * kHidden + ks * 16 + lg4]), acc);
    const float b2 = W.b2[n], w3 = from_bf16(W.w3[n]);
#pragma unroll
    for (int r = 0; r < 4; ++r) ps[r] = fmaf(fmaxf(acc[r] + b2, 0.f), w3, ps[r]);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) ps[r] += __shfl_xor(ps[r], off);
  if (li == 0)
#pragma unroll
    for (int r = 0; r < 4; ++r) S.part[wave][lg4 + r] = ps[r];
  __syncthreads();
  if (threadIdx.x < 16) {
    const int64_t row = row0 + threadIdx.x;
    const float sc = ((S.part[0][threadIdx.x] + S.part[1][threadIdx.x]) +
                      S.part[2][threadIdx.x]) + S.part[3][threadIdx.x];
    if (row < nrows) score[row] = sc + W.b3;
  }
}

// Scores of the active positions of every learned job, 16 per workgroup.
__global__ __launch_bounds__(256) void k_mlp(const JobDev* __restrict__ jobs, int njobs,
                                             const JobStep* __restrict__ js,
                                             const int32_t* __restrict__ pre) {
  __shared__ Mlp16Shared S;
  int jb, lb;
  if (!locate(pre, njobs, blockIdx.x, jb, lb)) return;
  const JobDev& J = jobs[jb];
  mlp16(*J.prop, S, J.feat, (int64_t)lb * 16, js[jb].m, J.score);
}

// Scores of `rows` feature rows (the C entry point), 16 per workgroup.
__global__ __launch_bounds__(256) void k_scores(const PropDev* __restrict__ W,
                                                const float* __restrict__ feat, int64_t rows,
                                                float* __restrict__ score) {
  __shared__ Mlp16Shared S;
  mlp16(*W, S, feat, (int64_t)blockIdx.x * 16, rows, score);
}

// ---------------------------------------------------------------------------
// top-K
// ---------------------------------------------------------------------------

// Order-preserving map of an FP32 score to 32 bits (NaN sorts lowest).
__device__ __forceinline__ uint32_t ord_f32(float f) {
  if (f != f) return 0u;
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// One workgroup per job: the K largest keys (score, then smaller original id)
// by an 8-bit radix select from the top byte; keys are distinct, so exactly K
// positions are at or above the K-th key.  Candidates are listed in
// ascending position order; cmark[p] = t + 1 marks them; ctrl->s_out is the
// best score outside them.
__global__ __launch_bounds__(1024) void k_topk(const JobDev* __restrict__ jobs, int njobs,
                                               const JobStep* __restrict__ js,
                                               const int32_t* __restrict__ pre, int t) {
  __shared__ uint32_t hist[256];
  __shared__ unsigned long long s_prefix;
  __shared__ int s_need, s_done;
  __shared__ int32_t scan[1024];
  __shared__ float smax[16];
  int jb, lb;
  if (!locate(pre, njobs, blockIdx.x, jb, lb)) return;
  const JobDev& J = jobs[jb];
  const int m = js[jb].m, K = js[jb].k;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto key = [&](int p) -> unsigned long long {
    return ((unsigned long long)ord_f32(J.score[p]) << 32) |
           (unsigned long long)(0xFFFFFFFFu - (uint32_t)J.act[p]);
  };
  // the need-th largest key: 8-bit radix passes from the top byte down
  auto select = [&](int need0) -> unsigned long long {
    __syncthreads();  // a previous select's readers are done with the shared state
    if (tid == 0) {
      s_prefix = 0ull;
      s_need = need0;
      s_done = 0;
    }
    unsigned long long prefix = 0ull, mask = 0ull;
    for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    if (tid < 256) hist[tid] = 0u;
    __syncthreads();
    for (int p = tid; p < m; p += 1024) {
      const unsigned long long k = key(p);
      if ((k & mask) == prefix) atomicAdd(&hist[(k >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (wave == 0) {
      // lane L holds bins 255 - 4L .. 252 - 4L (descending)
      uint32_t c[4], tot = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        c[i] = hist[255 - 4 * lane - i];
        tot += c[i];
      }
      uint32_t incl = tot;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
      }
      const int need = s_need;
      const unsigned long long bal = __ballot(incl >= (uint32_t)need);
      const int first = __ffsll((long long)bal) - 1;
      if (lane == first) {
        uint32_t excl = incl - tot;
        int dg = 255 - 4 * lane - 3;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (excl + c[i] >= (uint32_t)need) {
            dg = 255 - 4 * lane - i;
            break;
          }
          excl += c[i];
        }
        s_prefix = s_prefix | ((unsigned long long)dg << shift);
        s_need = need - (int)excl;
        // every key in this digit's bucket is needed: the K-th largest key
        // is at or above the prefix with the lower bits cleared
        if (hist[dg] == (uint32_t)(need - (int)excl)) s_done = 1;
      }
    }
    __syncthreads();
    prefix = s_prefix;
    mask |= 0xFFull << shift;
    if (s_done) break;
    }
    return prefix;
  };
  const unsigned long long prefix = select(K);
  // prefix is the K-th largest key; compact positions p with key(p) >= prefix
  const int per = (m + 1023) / 1024;
  const int p0 = tid * per, p1 = min(p0 + per, m);
  int cnt = 0;
  float best_out = -INFINITY;
  for (int p = p0; p < p1; ++p) {
    if (key(p) >= prefix) ++cnt;
    else best_out = fmaxf(best_out, J.score[p] == J.score[p] ? J.score[p] : -INFINITY);
  }
  scan[tid] = cnt;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t v = tid >= off ? scan[tid - off] : 0;
    __syncthreads();
    scan[tid] += v;
    __syncthreads();
  }
  int w = scan[tid] - cnt;
  for (int p = p0; p < p1; ++p)
    if (key(p) >= prefix) {
      if (w < K) J.cand[w] = p;
      J.cmark[p] = t + 1;
      ++w;
    }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) best_out = fmaxf(best_out, __shfl_xor(best_out, off));
  if (lane == 0) smax[wave] = best_out;
  __syncthreads();
  if (tid == 0) {
    float b = smax[0];
    for (int i = 1; i < 16; ++i) b = fmaxf(b, smax[i]);
    J.ctrl->s_out = b;
  }
  // extension list: the ne keys below the candidates' (keys are distinct, so
  // exactly ne positions lie in [pe, prefix)), ascending, padded with m
  const int ne = ext_count(m, K, J.ne_max);
  if (ne <= 0) return;  // workgroup-uniform
  const unsigned long long pe = select(K + ne);
  int ce = 0;
  for (int p = p0; p < p1; ++p) {
    const unsigned long long k = key(p);
    ce += (k >= pe && k < prefix) ? 1 : 0;
  }
  __syncthreads();
  scan[tid] = ce;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t v = tid >= off ? scan[tid - off] : 0;
    __syncthreads();
    scan[tid] += v;
    __syncthreads();
  }
  int we = scan[tid] - ce;
  for (int p = p0; p < p1; ++p) {
    const unsigned long long k = key(p);
    if (k >= pe && k < prefix) {
      if (we < ne) J.ext[we] = p;
      ++we;
    }
  }
  const int padded = cdiv(ne, kTileVars) * kTileVars;
  for (int c = ne + tid; c < padded; c += 1024) J.ext[c] = m;
}

// ---------------------------------------------------------------------------
// candidate rows of the measure
// ---------------------------------------------------------------------------

template <int W>
__global__ __launch_bounds__(64 * W) void k_pair_cand(const JobDev* __restrict__ jobs, int njobs,
                                                      const JobStep* __restrict__ js,
                                                      const int32_t* __restrict__ pre, int G) {
  pair_tiles<kModeCand, false, W>(jobs, njobs, js, pre, G);
}

// Witness pairs: one workgroup per non-candidate position l whose candidate
// bound lb[l] (from k_cand_k) does not exceed the best candidate's k (the
// others are bounded already).  For each of its kWit witnesses w (the most
// correlated other active variables, from k_features) that is not a
// candidate, the workgroup evaluates both residual directions of (l, w) over
// all samples with the hot loop's arithmetic (the eight waves take
// interleaved 64-sample blocks, the next block prefetched), reduces in FP64,
// and adds min(0, R(l, w))^2 (the share of k_l in that column) to lb[l].
constexpr int kWitWaves = 8;  // waves per witness workgroup

__global__ __launch_bounds__(64 * kWitWaves) void k_pair_wit(const JobDev* __restrict__ jobs,
                                                              int njobs,
                                                              const JobStep* __restrict__ js,
                                                              const int32_t* __restrict__ pre,
                                                              int t) {
  __shared__ double red[kWitWaves][4 * kWit];
  __shared__ double s_kb[kWitWaves];
  int jb, l;
  if (!locate(pre, njobs, blockIdx.x, jb, l)) return;
  const JobDev& J = jobs[jb];
  const int m = js[jb].m, K = js[jb].k;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (l >= m || J.cmark[l] == t + 1) return;  // workgroup-uniform
  // the best candidate's k
  double kb0 = INFINITY;
  for (int c = threadIdx.x; c < K; c += 64 * kWitWaves) kb0 = fmin(kb0, J.kc[c]);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) kb0 = fmin(kb0, __shfl_xor(kb0, off));
  if (lane == 0) s_kb[wave] = kb0;
  __syncthreads();
  double kbest = s_kb[0];
#pragma unroll
  for (int w = 1; w < kWitWaves; ++w) kbest = fmin(kbest, s_kb[w]);
  // bounded by the candidates alone (beyond the near-tie limit when near-ties
  // are decided in FP64, the suspects' threshold)
  if (J.lb[l] > (J.tie_on ? tie_limit(kbest) : kbest)) return;
  int wq[kWit];
  bool on[kWit];
  bool any = false;
#pragma unroll
  for (int q = 0; q < kWit; ++q) {
    const int w = J.wit[(int64_t)l * kWit + q];
    on[q] = w >= 0 && w < m && w != l && J.cmark[w] != t + 1;
    wq[q] = on[q] ? w : l;
    any |= on[q];
  }
  if (!any) return;
  // everything below up to the sample loop is workgroup-uniform: keep the
  // row bases and pair constants in SGPRs
  auto uni = [](float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
  };
  const int64_t ldz = J.ldz;
  const int sl = __builtin_amdgcn_readfirstlane(J.act[l]);
  const float* zl = J.z + (int64_t)sl * ldz;
  const float* zw[kWit];
  float kr[kWit], kh[kWit], kl[kWit];
#pragma unroll
  for (int q = 0; q < kWit; ++q) {
    const int sw = __builtin_amdgcn_readfirstlane(J.act[wq[q]]);
    zw[q] = J.z + (int64_t)sw * ldz;
    double r = on[q] ? J.rho[(int64_t)sl * J.d + sw] : 0.0;
    const double lim = 1.0 - kCollinear;
    r = r > lim ? lim : (r < -lim ? -lim : r);
    const double c1 = -2.0 * kLog2e / sqrt(1.0 - r * r);
    kr[q] = uni((float)r);
    kh[q] = uni((float)c1);
    kl[q] = uni((float)(c1 - (double)(float)c1));
  }
  // dir 0: residual of l on w; dir 1: residual of w on l
  float P0[kWit], A0[kWit], B0[kWit], P1[kWit], A1[kWit], B1[kWit];
#pragma unroll
  for (int q = 0; q < kWit; ++q) {
    P0[q] = P1[q] = 1.f;
    A0[q] = A1[q] = -kS1Start;
    B0[q] = B1[q] = 0.f;
  }
  const int nk = J.n_pad / 64;  // 64-sample blocks; this wave takes k = wave, wave + kWitWaves, ...
  int k = wave;
  float x = 0.f, y[kWit];
#pragma unroll
  for (int q = 0; q < kWit; ++q) y[q] = 0.f;
  if (k < nk) {
    x = zl[k * 64 + lane];
#pragma unroll
    for (int q = 0; q < kWit; ++q) y[q] = zw[q][k * 64 + lane];
  }
  int kb = 0;
  for (; k < nk; k += kWitWaves) {
    const bool more = k + kWitWaves < nk;
    const int s1 = (more ? k + kWitWaves : k) * 64 + lane;  // the last block re-reads itself
    const float nx = zl[s1];
    float ny[kWit];
#pragma unroll
    for (int q = 0; q < kWit; ++q) ny[q] = zw[q][s1];
#pragma unroll
    for (int q = 0; q < kWit; ++q) {
      eval_dir(x, y[q], kr[q], kh[q], kl[q], P0[q], A0[q], B0[q]);
      eval_dir(y[q], x, kr[q], kh[q], kl[q], P1[q], A1[q], B1[q]);
    }
    if (++kb == kLogBlock || !more) {
      const float off = 1.5f * (float)kb;  // exact
#pragma unroll
      for (int q = 0; q < kWit; ++q) {
        A0[q] += __builtin_amdgcn_logf(P0[q]) - off;
        A1[q] += __builtin_amdgcn_logf(P1[q]) - off;
        P0[q] = P1[q] = 1.f;
      }
      kb = 0;
    }
    x = nx;
#pragma unroll
    for (int q = 0; q < kWit; ++q) y[q] = ny[q];
  }
  // FP64 wave sums, one witness at a time (few registers live at once)
#pragma unroll
  for (int q = 0; q < kWit; ++q) {
    double v[4] = {(double)A0[q], (double)B0[q], (double)A1[q], (double)B1[q]};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v[i] += __shfl_xor(v[i], off);
    }
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) red[wave][4 * q + i] = v[i];
    }
  }
  __syncthreads();
  if (threadIdx.x >= kWit) return;
  const int q = threadIdx.x;  // lanes 0 .. kWit-1 of wave 0, one witness each
  double res = 0.0;
#pragma unroll
  for (int h = 0; h < kWit; ++h) {
    if (h != q || !on[h]) continue;
    double sm[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      sm[c] = red[0][4 * h + c];
#pragma unroll
      for (int w = 1; w < kWitWaves; ++w) sm[c] += red[w][4 * h + c];
    }
    const int sw = J.act[wq[h]];
    double r = J.rho[(int64_t)sl * J.d + sw];
    const double lim = 1.0 - kCollinear;
    r = r > lim ? lim : (r < -lim ? -lim : r);
    const double al = 1.0 / sqrt(1.0 - r * r);
    // every lane of the workgroup started its log cosh sum at -kS1Start
    const double bias = 64.0 * kWitWaves * (double)kS1Start + 0.5 * (double)J.n_pad;
    const double inv_n = 1.0 / (double)J.n;
    const double h_lw = entropy_from_moments(kLn2 * (sm[0] + bias) * inv_n, al * sm[1] * inv_n);
    const double h_wl = entropy_from_moments(kLn2 * (sm[2] + bias) * inv_n, al * sm[3] * inv_n);
    const double R = (J.hm[sw] + h_lw) - (J.hm[sl] + h_wl);
    res = R < 0.0 ? R * R : 0.0;
  }
  // lanes 0 .. kWit-1 of wave 0 hold the terms: lane 0 adds them in order
  double tot = res;
#pragma unroll
  for (int h = 1; h < kWit; ++h) tot += __shfl(res, h, 64);
  if (q == 0) J.lb[l] += tot;
}

// R(c, j) for candidate c against every active position j (0 for j = c),
// stored rc[c * d + j].  Same arithmetic as the all-pairs combine.
__global__ __launch_bounds__(256) void k_combine_cand(const JobDev* __restrict__ jobs, int njobs,
                                                      const JobStep* __restrict__ js,
                                                      const int32_t* __restrict__ pre) {
  int jb, lb;
  if (!locate(pre, njobs, blockIdx.x, jb, lb)) return;
  const JobDev& J = jobs[jb];
  const JobStep S = js[jb];
  const int gid = lb * 256 + threadIdx.x;
  if (gid >= S.nct * 64) return;
  const int tile = gid >> 6, wave = (gid >> 4) & 3, q = gid & 15;
  const int bi = tile / S.nblk, bj = tile - bi * S.nblk;
  const int wi = wave >> 1, wj = wave & 1;
  const int m = S.m;
  const int ci = bi * kTileVars + wi * kWaveVars + (q >> 2);
  const int pj = bj * kTileVars + wj * kWaveVars + (q & 3);
  if (pj >= m) return;
  const int pi = J.cand[ci];
  double* out = J.rc + (int64_t)ci * J.d + pj;
  if (pi == pj) {
    *out = 0.0;
    return;
  }
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int sp = 0; sp < S.nsplit_c; ++sp) {
    const double* src = J.partc + (((int64_t)sp * S.nct + tile) * 4 + wave) * 64 + q * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] += src[c];
  }
  const double s1_bias = (double)S.nsplit_c * 64.0 * (double)kS1Start + 0.5 * (double)J.n_pad;
  const double inv_n = 1.0 / (double)J.n;
  const int si = J.act[pi], sj = J.act[pj];
  double r = J.rho[(int64_t)si * J.d + sj];
  const double lim = 1.0 - kCollinear;
  r = r > lim ? lim : (r < -lim ? -lim : r);
  const double al = 1.0 / sqrt(1.0 - r * r);
  const double h_ij = entropy_from_moments(kLn2 * (s[0] + s1_bias) * inv_n, al * s[1] * inv_n);
  const double h_ji = entropy_from_moments(kLn2 * (s[2] + s1_bias) * inv_n, al * s[3] * inv_n);
  *out = (J.hm[sj] + h_ij) - (J.hm[si] + h_ji);
}

// Exact k of every candidate (kc[c] = sum_j min(0, R(c, j))^2, one wave per
// candidate) and the lower bound of every other variable's k (lb[l] = sum_c
// max(0, R(c, l))^2, since R(l, c) = -R(c, l); +inf at candidate positions).
// One launch: the first workgroups (the row kind's schedule) do the rows, the
// rest (the column kind's) the columns; a column workgroup covers 64
// positions, wave w summing candidates c = w, w + 4, ... in a fixed order.
__global__ __launch_bounds__(256) void k_cand_k(const JobDev* __restrict__ jobs, int njobs,
                                                const JobStep* __restrict__ js,
                                                const int32_t* __restrict__ pre_row,
                                                const int32_t* __restrict__ pre_col, int t) {
  __shared__ double part[4][64];
  const int nrow = pre_row[njobs];
  int jb, lb;
  if (blockIdx.x < nrow) {
    if (!locate(pre_row, njobs, blockIdx.x, jb, lb)) return;
    const JobDev& J = jobs[jb];
    const int m = js[jb].m;
    const int lane = threadIdx.x & 63;
    const int c = lb * 4 + (threadIdx.x >> 6);
    if (c >= js[jb].k) return;
    const double* row = J.rc + (int64_t)c * J.d;
    double k = 0.0;
    for (int q = lane; q < m; q += 64) {
      const double x = row[q];
      const double ng = x < 0.0 ? x : 0.0;
      k += ng * ng;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) k += __shfl_xor(k, off);
    if (lane == 0) J.kc[c] = k;
    return;
  }
  if (!locate(pre_col, njobs, blockIdx.x - nrow, jb, lb)) return;
  const JobDev& J = jobs[jb];
  const int m = js[jb].m, K = js[jb].k;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l = lb * 64 + lane;
  double s = 0.0;
  if (l < m)
    for (int c = wave; c < K; c += 4) {
      const double x = J.rc[(int64_t)c * J.d + l];
      const double ps = x > 0.0 ? x : 0.0;
      s += ps * ps;
    }
  part[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && l < m)
    J.lb[l] = J.cmark[l] == t + 1 ? INFINITY
                                  : ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
}

// Best of a list of measured rows (-k, ties to the smaller original id),
// merged with `seed` (thread 0's value) and reduced over the 256 threads of a
// workgroup; valid in every thread.
__device__ inline Best best_of_rows(const double* __restrict__ kvals,
                                    const int32_t* __restrict__ pos, int count,
                                    const int32_t* __restrict__ act, Best seed, Best* sh) {
  const int tid = threadIdx.x;
  Best b = tid == 0 ? seed : Best{-INFINITY, 0x7fffffff, -1, -INFINITY};
  for (int c = tid; c < count; c += 256) {
    double v = -kvals[c];
    if (v != v) v = -INFINITY;
    const int p = pos[c];
    const Best x{v, act[p], p, -INFINITY};
    b = (b.pos < 0) ? x : merge(b, x);
  }
  sh[tid] = b;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      const Best o = sh[tid + off];
      if (o.pos >= 0) sh[tid] = (sh[tid].pos < 0) ? o : merge(sh[tid], o);
    }
    __syncthreads();
  }
  const Best r = sh[0];
  __syncthreads();
  return r;
}

// Commit the choice of a learned step exactly as the full selection does.
__device__ inline void commit_choice(const JobDev& J, int t, int m, const Best& best) {
  J.order[t] = best.slot;
  J.ctrl->exo_slot = best.slot;
  J.ctrl->exo_pos = best.pos;
  J.ctrl->full = 0;
  if (J.gaps) J.gaps[t] = best.v - best.v2;
  J.act[best.pos] = J.act[m - 1];
}

// Near-tie set of a learned decision (the full selection's rule): every row
// of the list (exact k values kv[c] of positions pos[c], c < n) whose k is
// at most lim, appended to J.tie through the shared counter *cnt.  Called by
// every thread of the workgroup.
__device__ inline void gather_ties(const JobDev& J, double lim, const double* kv,
                                   const int32_t* pos, int n, int* cnt) {
  for (int c = threadIdx.x; c < n; c += blockDim.x)
    if (kv[c] <= lim) {
      const int w = atomicAdd(cnt, 1);
      if (w < kMaxTie) J.tie[w] = pos[c];
    }
}

// The learned choice `best`, or (2 .. kMaxTie near-tied rows listed in
// J.tie) its deferral to the FP64 decision: the full step is gated off
// either way.  Thread 0 only.
__device__ inline void commit_or_defer(const JobDev& J, int t, int m, const Best& best,
                                       int ntie) {
  if (J.tie_on && ntie > kMaxTie) J.ctrl->n_tie_overflow += 1;
  if (J.tie_on && ntie >= 2 && ntie <= kMaxTie) {
    J.ctrl->ntie = ntie;
    J.ctrl->tie_t = t;
    J.ctrl->tie_done = 0;
    for (int r = 0; r < kMaxTie; ++r) J.ctrl->tie_row_done[r] = 0;
    J.ctrl->tie_audit = 0;
    J.ctrl->full = 0;
    if (J.gaps) J.gaps[t] = best.v - best.v2;
  } else {
    commit_choice(J, t, m, best);
  }
}

// The learned decision of one job (one workgroup).  Best candidate by -k with
// ties to the smaller original id.  Suspects: non-candidates whose lower bound
// does not exceed its k (only they could still win).  No suspect: certified,
// the choice is the plain one.  At most suspect_cap suspects: they are listed
// (ascending position, padded to a multiple of 8 with position m) for the
// second pass, which decides exactly.  More: accepted when its score leads
// every non-candidate's by at least delta, else the full step decides.  Audit
// and teacher-forced steps always hand the step to the full kernels.
__global__ __launch_bounds__(256) void k_lselect(const JobDev* __restrict__ jobs, int njobs,
                                                 const JobStep* __restrict__ js,
                                                 const int32_t* __restrict__ pre, int t) {
  __shared__ Best sh[256];
  __shared__ int shs[256];
  int jb, lb;
  if (!locate(pre, njobs, blockIdx.x, jb, lb)) return;
  const JobDev& J = jobs[jb];
  const int m = js[jb].m, K = js[jb].k;
  const int tid = threadIdx.x;
  const Best best =
      best_of_rows(J.kc, J.cand, K, J.act, Best{-INFINITY, 0x7fffffff, -1, -INFINITY}, sh);
  const double kbest = -best.v;
  // with the FP64 tie resolution, a variable whose k might come within the
  // near-tie limit of the best must have its exact row too
  const double lim = J.tie_on ? tie_limit(kbest) : kbest;
  auto suspect = [&](int l) {
    const double v = J.lb[l];
    return !(v == v && v > lim);  // NaN bounds count as suspects
  };
  // count, then (if listed) write in ascending position order: thread chunks
  const int per = (m + 255) / 256;
  const int p0 = tid * per, p1 = min(p0 + per, m);
  int mine = 0;
  for (int l = p0; l < p1; ++l) mine += suspect(l) ? 1 : 0;
  shs[tid] = mine;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int v = tid >= off ? shs[tid - off] : 0;
    __syncthreads();
    shs[tid] += v;
    __syncthreads();
  }
  const int nsus = shs[255];
  const bool certified = nsus == 0;
  const float margin = J.score[best.pos] - J.ctrl->s_out;
  const bool audit = J.audit_every > 0 && t % J.audit_every == 0;
  const bool forced = t < J.forced_len;  // teacher forcing is applied by the full step
  const bool handover = audit || forced;
  const bool expand = !handover && !certified && nsus <= suspect_cap(m, K, J.cap_s);
  const bool take = !handover && (certified || (!expand && margin >= J.delta));
  const bool fallback = !handover && !take && !expand;
  if (expand) {
    int w = shs[tid] - mine;
    for (int l = p0; l < p1; ++l)
      if (suspect(l)) J.cand2[w++] = l;
    const int padded = (nsus + kTileVars - 1) / kTileVars * kTileVars;
    for (int c = nsus + tid; c < padded; c += 256) J.cand2[c] = m;
  }
  if (J.measures && take) {
    double* row = J.measures + (int64_t)t * J.d;
    for (int v = tid; v < J.d; v += 256) row[v] = NAN;
    __syncthreads();
    for (int c = tid; c < K; c += 256) row[J.act[J.cand[c]]] = -J.kc[c];
  }
  // a certified choice goes to the FP64 decision when candidates tie with it
  // (a choice the margin accepted is not exact anyway)
  if (tid == 0) shs[0] = 0;
  __syncthreads();
  if (take && certified && J.tie_on) gather_ties(J, lim, J.kc, J.cand, K, &shs[0]);
  __syncthreads();
  const int ntie = certified ? shs[0] : 0;
  if (tid != 0) return;
  Ctrl* C = J.ctrl;
  C->full = 1;
  C->nsus = expand ? nsus : 0;
  C->learned_slot = best.slot;
  C->n_learned += 1;
  C->n_certified += certified ? 1 : 0;
  C->n_audit += audit ? 1 : 0;
  C->n_fallback += fallback ? 1 : 0;
  C->n_suspects_sum += nsus;
  if (nsus > C->n_suspects_max) C->n_suspects_max = nsus;
  if (J.steplog)
    J.steplog[t] = take ? 1 : (expand ? (4 | (nsus << 4)) : (audit ? 3 : 2));
  if (take) commit_or_defer(J, t, m, best, ntie);
}

// Plan of the second pass: per job, the suspects listed at this step (0 for
// jobs without a listing) and the prefix sums of its kinds.  Stage 0 plans
// the extension columns (kinds kKPairE .. kKCompE) for the suspects k_lselect
// listed; stage 1 the suspects' full rows (kKPairS .. kKLsel2) for those
// the extension left (or all listed, without extension columns), with the
// suspect pass's sample split from the batch's suspect items.
__global__ __launch_bounds__(1024) void k_susp_schedule(const JobDev* __restrict__ jobs,
                                                        int njobs, JobStep* __restrict__ js,
                                                        int32_t* __restrict__ pre, int stage,
                                                        int num_cu, Tune tu) {
  auto plan = [&](int j) -> long long {
    JobStep s = js[j];
    s.nsus = s.learned ? jobs[j].ctrl->nsus : 0;
    if (stage == 0) {
      s.ne = s.learned ? ext_count(s.m, s.k, jobs[j].ne_max) : 0;
      s.nct3 = s.ne > 0 ? cdiv(s.nsus, kTileVars) * cdiv(s.ne, kTileVars) : 0;
    } else {
      s.nct2 = cdiv(s.nsus, kTileVars) * s.nblk;
    }
    js[j] = s;
    return stage == 1 ? 2LL * s.nct2 : 0;
  };
  auto split = [&](int j, long long items_s) {
    if (stage != 1) return;
    JobStep s = js[j];
    job_split_susp(s, jobs[j].n_pad, items_s, num_cu, tu, jobs[j].tie_on != 0);
    js[j] = s;
  };
  const int k0 = stage == 0 ? kKPairE : kKPairS, k1 = stage == 0 ? kKCompE : kKLsel2;
  const int tid = threadIdx.x, lane = tid & 63;
  if (njobs <= 64) {  // one wave, no barriers
    if (tid >= 64) return;
    long long items = lane < njobs ? plan(lane) : 0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) items += __shfl_xor(items, off);
    if (lane < njobs) split(lane, items);
  } else {
    __shared__ long long items;
    if (tid == 0) items = 0;
    __syncthreads();
    long long mine = 0;
    for (int j = tid; j < njobs; j += 1024) mine += plan(j);
    if (mine) atomicAdd(reinterpret_cast<unsigned long long*>(&items), (unsigned long long)mine);
    __syncthreads();
    for (int j = tid; j < njobs; j += 1024) split(j, items);
    __syncthreads();
  }
  // prefix sums of the kinds: one wave per kind, 64 jobs at a time
  const int nwaves = njobs <= 64 ? 1 : 16;
  for (int kind = k0 + (tid >> 6); kind <= k1; kind += nwaves) {
    int32_t* out = pre + (int64_t)kind * (njobs + 1);
    int32_t run = 0;
    for (int j0 = 0; j0 < njobs; j0 += 64) {
      const int j = j0 + lane;
      const int32_t c = j < njobs ? kind_count(js[j], kind) : 0;
      int32_t incl = c;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int32_t o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
      }
      if (j < njobs) out[j] = run + incl - c;
      run += __shfl(incl, 63);
    }
    if (lane == 0) out[njobs] = run;
  }
}

// The bounded-grid pair kernels (suspect and extension rows) walk their items
// in a loop.
template <int W>
__global__ __launch_bounds__(64 * W) void k_pair_susp(const JobDev* __restrict__ jobs,
                                                         int njobs,
                                                         const JobStep* __restrict__ js,
                                                         const int32_t* __restrict__ pre,
                                                         int G) {
  pair_tiles<kModeSusp, true, W>(jobs, njobs, js, pre, G);
}

template <int W>
__global__ __launch_bounds__(64 * W) void k_pair_ext(const JobDev* __restrict__ jobs,
                                                        int njobs,
                                                        const JobStep* __restrict__ js,
                                                        const int32_t* __restrict__ pre,
                                                        int G) {
  pair_tiles<kModeExt, true, W>(jobs, njobs, js, pre, G);
}

// The extension columns' share of every listed suspect's k: one wave per
// suspect l sums min(0, R(l, j))^2 over the extension columns j that are
// neither l nor one of l's witnesses (those entered the bound already), in
// a fixed order, and adds it to lb[l].  R as in the other combines.
__global__ __launch_bounds__(256) void k_ext_bound(const JobDev* __restrict__ jobs, int njobs,
                                                   const JobStep* __restrict__ js,
                                                   const int32_t* __restrict__ pre) {
  for_blocks(pre, njobs, [&](int jb, int lb) {
    const JobDev& J = jobs[jb];
    const JobStep S = js[jb];
    const int lane = threadIdx.x & 63;
    const int ci = lb * 4 + (threadIdx.x >> 6);
    if (ci >= S.nsus) return;  // wave-uniform; no barriers below
    const int l = J.cand2[ci];
    const int sl = J.act[l];
    const int nbe = cdiv(S.ne, kTileVars);
    int wl[kWit];
#pragma unroll
    for (int q = 0; q < kWit; ++q) wl[q] = J.wit[(int64_t)l * kWit + q];
    const double s1_bias =
        (double)S.nsplit * 64.0 * (double)kS1Start + 0.5 * (double)J.n_pad;
    const double inv_n = 1.0 / (double)J.n;
    const double lim = 1.0 - kCollinear;
    double acc = 0.0;
    for (int e = lane; e < S.ne; e += 64) {
      const int j = J.ext[e];
      bool skip = j == l;
#pragma unroll
      for (int q = 0; q < kWit; ++q) skip |= j == wl[q];
      if (skip) continue;
      // the pair's slot in the extension pass's partial sums
      const int tile = (ci / kTileVars) * nbe + e / kTileVars;
      const int wave = ((ci % kTileVars) / kWaveVars) * 2 + (e % kTileVars) / kWaveVars;
      const int q = (ci % kWaveVars) * 4 + (e % kWaveVars);
      double sm[4] = {0.0, 0.0, 0.0, 0.0};
      for (int sp = 0; sp < S.nsplit; ++sp) {
        const double* src = J.parts + (((int64_t)sp * S.nct3 + tile) * 4 + wave) * 64 + q * 4;
#pragma unroll
        for (int c = 0; c < 4; ++c) sm[c] += src[c];
      }
      const int sj = J.act[j];
      double r = J.rho[(int64_t)sl * J.d + sj];
      r = r > lim ? lim : (r < -lim ? -lim : r);
      const double al = 1.0 / sqrt(1.0 - r * r);
      const double h_lj =
          entropy_from_moments(kLn2 * (sm[0] + s1_bias) * inv_n, al * sm[1] * inv_n);
      const double h_jl =
          entropy_from_moments(kLn2 * (sm[2] + s1_bias) * inv_n, al * sm[3] * inv_n);
      const double R = (J.hm[sj] + h_lj) - (J.hm[sl] + h_jl);
      if (R < 0.0) acc += R * R;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) J.lb[l] += acc;
  });
}

// Keep the listed suspects whose bound still does not exceed the best
// candidate's k (in place, ascending, padded with m); the count goes to
// ctrl->nsus for the rows pass.  None left: the best candidate is the exact
// choice and is committed here.
__global__ __launch_bounds__(256) void k_ext_compact(const JobDev* __restrict__ jobs, int njobs,
                                                     const JobStep* __restrict__ js,
                                                     const int32_t* __restrict__ pre, int t) {
  static_assert(kMaxSuspects <= 4 * 256, "four listed suspects per thread");
  __shared__ Best sh[256];
  __shared__ int shs[256];
  for_blocks(pre, njobs, [&](int jb, int) {
    const JobDev& J = jobs[jb];
    const JobStep S = js[jb];
    const int tid = threadIdx.x;
    const int m = S.m, n1 = S.nsus;
    const Best best =
        best_of_rows(J.kc, J.cand, S.k, J.act, Best{-INFINITY, 0x7fffffff, -1, -INFINITY}, sh);
    const double kbest = -best.v;
    const double lim = J.tie_on ? tie_limit(kbest) : kbest;
    const int per = (n1 + 255) / 256;
    const int c0 = min(tid * per, n1), c1 = min(c0 + per, n1);
    int v[4];
    bool keep[4];
    int mine = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int c = c0 + i;
      v[i] = c < c1 ? J.cand2[c] : 0;
      const double b = c < c1 ? J.lb[v[i]] : INFINITY;
      keep[i] = c < c1 && !(b == b && b > lim);  // NaN bounds stay suspects
      mine += keep[i] ? 1 : 0;
    }
    shs[tid] = mine;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int x = tid >= off ? shs[tid - off] : 0;
      __syncthreads();
      shs[tid] += x;
      __syncthreads();
    }
    const int n2 = shs[255];
    int w = shs[tid] - mine;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (keep[i]) J.cand2[w++] = v[i];
    const int padded = cdiv(n2, kTileVars) * kTileVars;
    for (int c = n2 + tid; c < padded; c += 256) J.cand2[c] = m;
    if (n2 == 0 && J.measures) {
      double* row = J.measures + (int64_t)t * J.d;
      for (int x = tid; x < J.d; x += 256) row[x] = NAN;
      __syncthreads();
      for (int c = tid; c < S.k; c += 256) row[J.act[J.cand[c]]] = -J.kc[c];
    }
    __syncthreads();
    if (tid == 0) shs[0] = 0;
    __syncthreads();
    if (n2 == 0 && J.tie_on) gather_ties(J, lim, J.kc, J.cand, S.k, &shs[0]);
    __syncthreads();
    const int ntie = shs[0];
    if (tid == 0) {
      Ctrl* C = J.ctrl;
      C->nsus = n2;
      if (n2 == 0) {
        C->n_expanded += 1;
        C->n_cleared += 1;
        commit_or_defer(J, t, m, best, ntie);
      }
    }
    __syncthreads();
  });
}

// R(s, j) of every listed suspect against every active position (0 for j = s).
__global__ __launch_bounds__(256) void k_combine_susp(const JobDev* __restrict__ jobs, int njobs,
                                                      const JobStep* __restrict__ js,
                                                      const int32_t* __restrict__ pre) {
  for_blocks(pre, njobs, [&](int jb, int lb) {
    const JobDev& J = jobs[jb];
    const JobStep S = js[jb];
    const int gid = lb * 256 + threadIdx.x;
    if (gid >= S.nct2 * 64) return;
    const int tile = gid >> 6, wave = (gid >> 4) & 3, q = gid & 15;
    const int bi = tile / S.nblk, bj = tile - bi * S.nblk;
    const int wi = wave >> 1, wj = wave & 1;
    const int m = S.m;
    const int ci = bi * kTileVars + wi * kWaveVars + (q >> 2);
    const int pj = bj * kTileVars + wj * kWaveVars + (q & 3);
    if (ci >= S.nsus || pj >= m) return;
    const int pi = J.cand2[ci];
    double* out = J.rc2 + (int64_t)ci * J.d + pj;
    if (pi == pj) {
      *out = 0.0;
      return;
    }
    double sm[4] = {0.0, 0.0, 0.0, 0.0};
    for (int sp = 0; sp < S.nsplit_s; ++sp) {
      const double* src = J.parts + (((int64_t)sp * S.nct2 + tile) * 4 + wave) * 64 + q * 4;
#pragma unroll
      for (int c = 0; c < 4; ++c) sm[c] += src[c];
    }
    const double s1_bias =
        (double)S.nsplit_s * 64.0 * (double)kS1Start + 0.5 * (double)J.n_pad;
    const double inv_n = 1.0 / (double)J.n;
    const int si = J.act[pi], sj = J.act[pj];
    double r = J.rho[(int64_t)si * J.d + sj];
    const double lim = 1.0 - kCollinear;
    r = r > lim ? lim : (r < -lim ? -lim : r);
    const double al = 1.0 / sqrt(1.0 - r * r);
    const double h_ij =
        entropy_from_moments(kLn2 * (sm[0] + s1_bias) * inv_n, al * sm[1] * inv_n);
    const double h_ji =
        entropy_from_moments(kLn2 * (sm[2] + s1_bias) * inv_n, al * sm[3] * inv_n);
    *out = (J.hm[sj] + h_ij) - (J.hm[si] + h_ji);
  });
}

// kc2[s] = sum_j min(0, R(s, j))^2, one wave per listed suspect.
__global__ __launch_bounds__(256) void k_susp_rowk(const JobDev* __restrict__ jobs, int njobs,
                                                   const JobStep* __restrict__ js,
                                                   const int32_t* __restrict__ pre) {
  for_blocks(pre, njobs, [&](int jb, int lb) {
    const JobDev& J = jobs[jb];
    const JobStep S = js[jb];
    const int lane = threadIdx.x & 63;
    const int c = lb * 4 + (threadIdx.x >> 6);
    if (c >= S.nsus) return;
    const double* row = J.rc2 + (int64_t)c * J.d;
    double k = 0.0;
    for (int q = lane; q < S.m; q += 64) {
      const double x = row[q];
      const double ng = x < 0.0 ? x : 0.0;
      k += ng * ng;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) k += __shfl_xor(k, off);
    if (lane == 0) J.kc2[c] = k;
  });
}

// The exact decision after the second pass: the best of candidates and
// suspects is the plain choice (every other variable's bound exceeds the
// best candidate's k, which is at least the new best's).
__global__ __launch_bounds__(256) void k_lselect2(const JobDev* __restrict__ jobs, int njobs,
                                                  const JobStep* __restrict__ js,
                                                  const int32_t* __restrict__ pre, int t) {
  __shared__ Best sh[256];
  __shared__ int s_tie;
  for_blocks(pre, njobs, [&](int jb, int) {
    const JobDev& J = jobs[jb];
    const JobStep S = js[jb];
    const int tid = threadIdx.x;
    Best b = best_of_rows(J.kc, J.cand, S.k, J.act,
                          Best{-INFINITY, 0x7fffffff, -1, -INFINITY}, sh);
    b = best_of_rows(J.kc2, J.cand2, S.nsus, J.act, b, sh);
    if (tid == 0) s_tie = 0;
    __syncthreads();
    if (J.tie_on) {
      const double lim = tie_limit(-b.v);
      gather_ties(J, lim, J.kc, J.cand, S.k, &s_tie);
      gather_ties(J, lim, J.kc2, J.cand2, S.nsus, &s_tie);
    }
    __syncthreads();
    const int ntie = s_tie;
    if (J.measures) {
      double* row = J.measures + (int64_t)t * J.d;
      for (int v = tid; v < J.d; v += 256) row[v] = NAN;
      __syncthreads();
      for (int c = tid; c < S.k; c += 256) row[J.act[J.cand[c]]] = -J.kc[c];
      for (int c = tid; c < S.nsus; c += 256) row[J.act[J.cand2[c]]] = -J.kc2[c];
    }
    __syncthreads();
    if (tid == 0) {
      J.ctrl->n_expanded += 1;
      J.ctrl->n_rows_sum += S.nsus;
      if (J.steplog) J.steplog[t] |= S.nsus << 16;
      commit_or_defer(J, t, S.m, b, ntie);
    }
    __syncthreads();
  });
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------

// Forward pass over the training rows with saved activations.
__global__ __launch_bounds__(256) void k_train_fwd(const PropDev* __restrict__ W,
                                                   const float* __restrict__ feat, int64_t rows,
                                                   float* __restrict__ score,
                                                   uint16_t* __restrict__ H1,
                                                   float* __restrict__ H2) {
  __shared__ MlpShared S;
  stage_w2(*W, S);
  __syncthreads();
  mlp_tile(*W, S, feat, (int64_t)blockIdx.x * 64, rows, score, H1, H2);
}

// Listwise softmax cross-entropy, one workgroup per list:
// loss_L = logsumexp(s_L) - s_target, ds = (softmax - onehot) / n_lists.
// A list outside [0, rows] or a target outside its list sets *status = 1 and
// contributes nothing.
// With `weights` (soft targets) the target distribution of list L is
// q = weights / sum(weights) over its rows and `targets` is not read; the
// loss is sum_r q_r (logsumexp(s) - s_r) and ds = (softmax(s) - q) / n_lists.
// Negative or non-finite weights, or a list whose weights sum to 0, set the
// status like a malformed list.
__global__ __launch_bounds__(256) void k_list_ce(const float* __restrict__ score, int64_t rows,
                                                 const int64_t* __restrict__ offsets,
                                                 const int64_t* __restrict__ targets,
                                                 const float* __restrict__ weights,
                                                 int n_lists, float* __restrict__ ds,
                                                 double* __restrict__ loss_part,
                                                 int32_t* __restrict__ status) {
  __shared__ double sh[256];
  __shared__ int s_bad;
  const int L = blockIdx.x;
  const int64_t a = offsets[L], b = offsets[L + 1];
  const int tid = threadIdx.x;
  const int64_t tg = weights ? a : targets[L];
  bool bad = !(0 <= a && a <= b && b <= rows && a <= tg && tg < b);
  double wsum = 0.0;
  if (weights && !bad) {
    if (tid == 0) s_bad = 0;
    __syncthreads();
    double loc = 0.0;
    for (int64_t r = a + tid; r < b; r += 256) {
      const float w = weights[r];
      if (!(w >= 0.f) || !isfinite(w)) s_bad = 1;
      loc += (double)w;
    }
    wsum = block_sum_256(loc, sh);  // synchronizes: s_bad is final
    bad = s_bad != 0 || !(wsum > 0.0);
  }
  if (bad) {
    if (tid == 0) {
      *status = 1;
      loss_part[L] = 0.0;
    }
    return;
  }
  double mx = -INFINITY;
  for (int64_t r = a + tid; r < b; r += 256) mx = fmax(mx, (double)score[r]);
  sh[tid] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) sh[tid] = fmax(sh[tid], sh[tid + off]);
    __syncthreads();
  }
  mx = sh[0];
  __syncthreads();
  double se = 0.0;
  for (int64_t r = a + tid; r < b; r += 256) se += exp((double)score[r] - mx);
  const double tot = block_sum_256(se, sh);
  const double inv = 1.0 / (double)n_lists;
  const double lse = mx + log(tot);
  if (weights) {
    double qs = 0.0;  // sum_r q_r s_r
    for (int64_t r = a + tid; r < b; r += 256) {
      const double q = (double)weights[r] / wsum;
      const double p = exp((double)score[r] - mx) / tot;
      ds[r] = (float)((p - q) * inv);
      qs += q * (double)score[r];
    }
    qs = block_sum_256(qs, sh);
    if (tid == 0) loss_part[L] = lse - qs;
    return;
  }
  for (int64_t r = a + tid; r < b; r += 256) {
    const double p = exp((double)score[r] - mx) / tot;
    ds[r] = (float)((p - (r == tg ? 1.0 : 0.0)) * inv);
  }
  if (tid == 0) loss_part[L] = lse - (double)score[tg];
}

__global__ void k_zero_f32(float* __restrict__ p, int64_t n, int32_t* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
  if (i == 0 && status) *status = 0;
}

// LDS of the backward pass of one 64-row tile.
struct BwdShared {
  uint16_t w2t[kHidden][kLdW];  // W2^T[g][h] = W2[h][g]
  uint16_t dh2t[kHidden][kLdR]; // dh2^T[h][i] (BF16)
  uint16_t h1t[kHidden][kLdR];  // h1^T[g][i]
  uint16_t dh1t[kHidden][kLdR]; // dh1^T[g][i]
  uint16_t xt[kFeat][kLdR];     // x^T[f][i]
  float ds[64];
};

// Backward pass.  Each workgroup walks 64-row tiles (grid stride) and keeps its
// share of the weight gradients in registers (W2: wave w owns rows
// 32 w .. 32 w + 31 of dW2; W1: wave w owns rows 32 w .. + 31 of dW1) and
// the vector gradients in per-thread registers (thread h < 128), then writes
// one partial gradient of kParams values per workgroup.
__global__ __launch_bounds__(256) void k_train_bwd(const PropDev* __restrict__ W,
                                                   const float* __restrict__ feat, int64_t rows,
                                                   const float* __restrict__ dsv,
                                                   const uint16_t* __restrict__ H1,
                                                   const float* __restrict__ H2,
                                                   float* __restrict__ part) {
  __shared__ BwdShared S;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lg4 = (lane >> 4) * 4;
  for (int i = tid; i < kHidden * kHidden; i += 256) {
    const int h = i / kHidden, g = i % kHidden;
    S.w2t[g][h] = W->w2[i];
  }
  f32x4_t gw2[2][8];
  f32x4_t gw1[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    gw1[a] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 8; ++b) gw2[a][b] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  }
  float g_w3 = 0.f, g_b2 = 0.f, g_b1 = 0.f, g_b3 = 0.f;
  const int h_own = tid & (kHidden - 1);  // threads h and h + 128 split the rows
  const int half = tid >> 7;
  const float w3h = from_bf16(W->w3[h_own]);
  const int64_t ntile = (rows + 63) / 64;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t row0 = tile * 64;
    __syncthreads();
    if (tid < 64) S.ds[tid] = row0 + tid < rows ? dsv[row0 + tid] : 0.f;
    // x^T (BF16, normalized) and h1^T of the tile
    for (int e = tid; e < 64 * kFeat; e += 256) {
      const int i = e / kFeat, f = e % kFeat;
      const int64_t row = row0 + i;
      const float v = row < rows ? (feat[row * kFeat + f] - W->mu[f]) / W->sd[f] : 0.f;
      S.xt[f][i] = to_bf16(v);
    }
    for (int e = tid; e < 64 * kHidden; e += 256) {
      const int i = e / kHidden, g = e % kHidden;
      const int64_t row = row0 + i;
      S.h1t[g][i] = row < rows ? H1[row * kHidden + g] : (uint16_t)0;
    }
    __syncthreads();
    // dh2 = ds * w3 * [h2 > 0]; vector gradients of w3, b2, b3
    for (int i = half * 32; i < half * 32 + 32; ++i) {
      const int64_t row = row0 + i;
      float d = 0.f;
      if (row < rows) {
        const float h2 = H2[row * kHidden + h_own];
        const float dsi = S.ds[i];
        g_w3 = fmaf(dsi, h2, g_w3);
        d = h2 > 0.f ? dsi * w3h : 0.f;
        g_b2 += d;
      }
      S.dh2t[h_own][i] = to_bf16(d);
    }
    if (tid == 0)
      for (int i = 0; i < 64; ++i) g_b3 += S.ds[i];
    __syncthreads();
    // dh1 = (dh2 W2) * [h1 > 0]: rows 16 wave .. + 15, all 128 columns
#pragma unroll 1
    for (int nt = 0; nt < kHidden / 16; ++nt) {
      f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < kHidden / 16; ++ks) {
        // A[i][h] = dh2[i][h] = dh2t[h][i]; B[h][g] = W2[h][g] = w2t[g][h]
        bf16x4_t a;
#pragma unroll
        for (int j = 0; j < 4; ++j) a[j] = (short)S.dh2t[ks * 16 + lg4 + j][wave * 16 + li];
        const bf16x4_t b = load4(&S.w2t[nt * 16 + li][ks * 16 + lg4]);
        acc = mfma16(a, b, acc);
      }
      const int g = nt * 16 + li;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wave * 16 + lg4 + r;
        const float v = (S.h1t[g][i] & 0x7FFF) != 0 ? acc[r] : 0.f;  // h1 > 0 <=> a1 > 0
        S.dh1t[g][i] = to_bf16(v);
      }
    }
    __syncthreads();
    // b1 from the BF16 dh1 (as the weight gradient sees it)
    for (int i = half * 32; i < half * 32 + 32; ++i) g_b1 += from_bf16(S.dh1t[h_own][i]);
    // dW2[h][g] += sum_i dh2[i][h] h1[i][g]: wave owns h = 32 wave .. + 31
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int h = wave * 32 + a * 16 + li;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const bf16x4_t A = load4(&S.dh2t[h][ks * 16 + lg4]);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const bf16x4_t B = load4(&S.h1t[b * 16 + li][ks * 16 + lg4]);
          gw2[a][b] = mfma16(A, B, gw2[a][b]);
        }
      }
      // dW1[h][f] += sum_i dh1[i][h] x[i][f]
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const bf16x4_t A = load4(&S.dh1t[h][ks * 16 + lg4]);
        const bf16x4_t B = load4(&S.xt[li][ks * 16 + lg4]);
        gw1[a] = mfma16(A, B, gw1[a]);
      }
    }
  }
  // partial gradient of this workgroup
  float* out = part + (int64_t)blockIdx.x * kParams;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int h = wave * 32 + a * 16 + lg4 + r;
#pragma unroll
      for (int b = 0; b < 8; ++b) out[kOffW2 + h * kHidden + b * 16 + li] = gw2[a][b][r];
      out[kOffW1 + h * kFeat + li] = gw1[a][r];
    }
  }
  // the two halves of the vector gradients
  __shared__ float vec[3][256];
  vec[0][tid] = g_w3;
  vec[1][tid] = g_b2;
  vec[2][tid] = g_b1;
  __syncthreads();
  if (tid < kHidden) {
    out[kOffW3 + tid] = vec[0][tid] + vec[0][tid + 128];
    out[kOffB2 + tid] = vec[1][tid] + vec[1][tid + 128];
    out[kOffB1 + tid] = vec[2][tid] + vec[2][tid + 128];
  }
  if (tid == 0) out[kOffB3] = g_b3;
}

// grad[p] = sum over workgroups of the partials (fixed order); loss = mean.
__global__ __launch_bounds__(256) void k_grad_reduce(const float* __restrict__ part, int nparts,
                                                     float* __restrict__ grad,
                                                     const double* __restrict__ loss_part,
                                                     int n_lists, float* __restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < kParams) {
    double s = 0.0;
    for (int k = 0; k < nparts; ++k) s += (double)part[(int64_t)k * kParams + p];
    grad[p] = (float)s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && loss) {
    double s = 0.0;
    for (int L = 0; L < n_lists; ++L) s += loss_part[L];
    *loss = (float)(s / (double)n_lists);
  }
}

// Adam on the FP32 master weights (after the 32 normalisation values).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ prop,
                                              const float* __restrict__ grad,
                                              float* __restrict__ mom1, float* __restrict__ mom2,
                                              float lr, float beta1, float beta2, float eps,
                                              float c1, float c2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kParams) return;
  const float g = grad[p];
  const float m1 = beta1 * mom1[p] + (1.f - beta1) * g;
  const float m2 = beta2 * mom2[p] + (1.f - beta2) * g * g;
  mom1[p] = m1;
  mom2[p] = m2;
  prop[kPropNorm + p] -= lr * (m1 * c1) / (sqrtf(m2 * c2) + eps);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

static inline const int32_t* pre_kind(SchedDev sc, int njobs, int kind) {
  return sc.pre + (int64_t)kind * (njobs + 1);
}

hipError_t launch_prop_prep(const float* in, PropDev* out, const JobDev* jobs, int njobs,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_prop_prep, dim3(1), dim3(256), 0, st, in, out, jobs, njobs,
                     (int32_t*)nullptr);
  return hipGetLastError();
}

hipError_t launch_learned_front(const JobDev* jobs, int njobs, int t, SchedDev sc,
                                const int32_t* grid, hipStream_t st) {
  const JobStep* js = sc.js;
  if (grid[kKFeat] > 0)
    hipLaunchKernelGGL(k_features, dim3((unsigned)grid[kKFeat]), dim3(256), 0, st, jobs, njobs,
                       js, pre_kind(sc, njobs, kKFeat), t);
  if (grid[kKMlp] <= 0) return hipGetLastError();
  hipLaunchKernelGGL(k_mlp, dim3((unsigned)grid[kKMlp]), dim3(256), 0, st, jobs, njobs, js,
                     pre_kind(sc, njobs, kKMlp));
  hipLaunchKernelGGL(k_topk, dim3((unsigned)grid[kKTopk]), dim3(1024), 0, st, jobs, njobs, js,
                     pre_kind(sc, njobs, kKTopk), t);
  return hipGetLastError();
}

// The row kernels at 1, 2 or 4 waves per workgroup.
#define LG_LAUNCH_W(kern, waves, grid, st, ...)                                          \
  do {                                                                                   \
    if ((waves) == 1)                                                                    \
      hipLaunchKernelGGL(kern<1>, dim3((unsigned)(grid)), dim3(64), 0, st, __VA_ARGS__);  \
    else if ((waves) == 2)                                                               \
      hipLaunchKernelGGL(kern<2>, dim3((unsigned)(grid)), dim3(128), 0, st, __VA_ARGS__); \
    else                                                                                 \
      hipLaunchKernelGGL(kern<4>, dim3((unsigned)(grid)), dim3(256), 0, st, __VA_ARGS__); \
  } while (0)

hipError_t launch_pair_cand(const JobDev* jobs, int njobs, SchedDev sc, int grid, int waves,
                            hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  LG_LAUNCH_W(k_pair_cand, waves, grid, st, jobs, njobs, (const JobStep*)sc.js,
              pre_kind(sc, njobs, kKPairC), grid);
  return hipGetLastError();
}

hipError_t launch_learned_back(const JobDev* jobs, int njobs, int t, SchedDev sc,
                               const int32_t* grid, hipStream_t st) {
  const JobStep* js = sc.js;
  if (grid[kKLsel] <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine_cand, dim3((unsigned)grid[kKCombC]), dim3(256), 0, st, jobs,
                     njobs, js, pre_kind(sc, njobs, kKCombC));
  hipLaunchKernelGGL(k_cand_k, dim3((unsigned)(grid[kKRowkC] + grid[kKColC])), dim3(256), 0, st,
                     jobs, njobs, js, pre_kind(sc, njobs, kKRowkC), pre_kind(sc, njobs, kKColC),
                     t);
  if (grid[kKWit] > 0)
    hipLaunchKernelGGL(k_pair_wit, dim3((unsigned)grid[kKWit]), dim3(64 * kWitWaves), 0, st,
                       jobs, njobs,
                       js, pre_kind(sc, njobs, kKWit), t);
  hipLaunchKernelGGL(k_lselect, dim3((unsigned)grid[kKLsel]), dim3(256), 0, st, jobs, njobs, js,
                     pre_kind(sc, njobs, kKLsel), t);
  return hipGetLastError();
}

hipError_t launch_susp_schedule(const JobDev* jobs, int njobs, SchedDev sc, int stage,
                                int num_cu, Tune tu, hipStream_t st) {
  hipLaunchKernelGGL(k_susp_schedule, dim3(1), dim3(1024), 0, st, jobs, njobs, sc.js, sc.pre,
                     stage, num_cu, tu);
  return hipGetLastError();
}

hipError_t launch_pair_ext(const JobDev* jobs, int njobs, SchedDev sc, int grid, int waves,
                           hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  LG_LAUNCH_W(k_pair_ext, waves, grid, st, jobs, njobs, (const JobStep*)sc.js,
              pre_kind(sc, njobs, kKPairE), grid);
  return hipGetLastError();
}

hipError_t launch_ext_back(const JobDev* jobs, int njobs, int t, SchedDev sc, int g_bound,
                           int g_comp, hipStream_t st) {
  if (g_comp <= 0) return hipSuccess;
  const JobStep* js = sc.js;
  hipLaunchKernelGGL(k_ext_bound, dim3((unsigned)g_bound), dim3(256), 0, st, jobs, njobs, js,
                     pre_kind(sc, njobs, kKBoundE));
  hipLaunchKernelGGL(k_ext_compact, dim3((unsigned)g_comp), dim3(256), 0, st, jobs, njobs, js,
                     pre_kind(sc, njobs, kKCompE), t);
  return hipGetLastError();
}

hipError_t launch_pair_susp(const JobDev* jobs, int njobs, SchedDev sc, int grid, int waves,
                            hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  LG_LAUNCH_W(k_pair_susp, waves, grid, st, jobs, njobs, (const JobStep*)sc.js,
              pre_kind(sc, njobs, kKPairS), grid);
  return hipGetLastError();
}

hipError_t launch_susp_back(const JobDev* jobs, int njobs, int t, SchedDev sc, int g_comb,
                            int g_rowk, int g_sel, hipStream_t st) {
  const JobStep* js = sc.js;
  if (g_sel <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine_susp, dim3((unsigned)g_comb), dim3(256), 0, st, jobs, njobs, js,
                     pre_kind(sc, njobs, kKCombS));
  hipLaunchKernelGGL(k_susp_rowk, dim3((unsigned)g_rowk), dim3(256), 0, st, jobs, njobs, js,
                     pre_kind(sc, njobs, kKRowkS));
  hipLaunchKernelGGL(k_lselect2, dim3((unsigned)g_sel), dim3(256), 0, st, jobs, njobs, js,
                     pre_kind(sc, njobs, kKLsel2), t);
  return hipGetLastError();
}

// Training workspace: [status][PropDev][score f32 rows][ds f32 rows][H1 u16 rows*128]
// [H2 f32 rows*128][loss_part f64 n_lists][partials f32 nparts*kParams]
TrainLayout make_train_layout(int64_t rows, int32_t n_lists) {
  TrainLayout T{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) & ~size_t(255);
    return o;
  };
  T.rows = rows;
  T.n_lists = n_lists;
  const int64_t ntile = (rows + 63) / 64;
  T.nparts = (int)(ntile < kTrainParts ? ntile : kTrainParts);
  T.status = take(sizeof(int32_t));
  T.prop = take(sizeof(PropDev));
  T.score = take(sizeof(float) * (size_t)rows);
  T.ds = take(sizeof(float) * (size_t)rows);
  T.h1 = take(sizeof(uint16_t) * (size_t)rows * kHidden);
  T.h2 = take(sizeof(float) * (size_t)rows * kHidden);
  T.loss_part = take(sizeof(double) * (size_t)n_lists);
  T.part = take(sizeof(float) * (size_t)T.nparts * kParams);
  T.total = off;
  return T;
}

hipError_t launch_scores(const float* prop, const float* feat, int64_t rows, float* score,
                         char* ws, hipStream_t st) {
  PropDev* W = reinterpret_cast<PropDev*>(ws);
  hipLaunchKernelGGL(k_prop_prep, dim3(1), dim3(256), 0, st, prop, W, (const JobDev*)nullptr, 0,
                     (int32_t*)nullptr);
  hipLaunchKernelGGL(k_scores, dim3((unsigned)((rows + 15) / 16)), dim3(256), 0, st,
                     (const PropDev*)W, feat, rows, score);
  return hipGetLastError();
}

hipError_t launch_grad(const TrainLayout& T, const float* prop, const float* feat,
                       const int64_t* offsets, const int64_t* targets, const float* weights,
                       float* grad, float* loss, float* score_out, char* ws, hipStream_t st) {
  PropDev* W = reinterpret_cast<PropDev*>(ws + T.prop);
  float* score = reinterpret_cast<float*>(ws + T.score);
  float* ds = reinterpret_cast<float*>(ws + T.ds);
  uint16_t* H1 = reinterpret_cast<uint16_t*>(ws + T.h1);
  float* H2 = reinterpret_cast<float*>(ws + T.h2);
  double* lp = reinterpret_cast<double*>(ws + T.loss_part);
  float* part = reinterpret_cast<float*>(ws + T.part);
  int32_t* status = reinterpret_cast<int32_t*>(ws + T.status);
  hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)((T.rows + 255) / 256)), dim3(256), 0, st, ds,
                     T.rows, status);
  hipLaunchKernelGGL(k_prop_prep, dim3(1), dim3(256), 0, st, prop, W, (const JobDev*)nullptr, 0,
                     status);
  const int64_t ntile = (T.rows + 63) / 64;
  hipLaunchKernelGGL(k_train_fwd, dim3((unsigned)ntile), dim3(256), 0, st, (const PropDev*)W,
                     feat, T.rows, score, H1, H2);
  hipLaunchKernelGGL(k_list_ce, dim3((unsigned)T.n_lists), dim3(256), 0, st,
                     (const float*)score, T.rows, offsets, targets, weights, T.n_lists, ds, lp,
                     status);
  hipLaunchKernelGGL(k_train_bwd, dim3((unsigned)T.nparts), dim3(256), 0, st, (const PropDev*)W,
                     feat, T.rows, (const float*)ds, (const uint16_t*)H1, (const float*)H2,
                     part);
  hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)((kParams + 255) / 256)), dim3(256), 0, st,
                     (const float*)part, T.nparts, grad, (const double*)lp, T.n_lists, loss);
  if (score_out)
    return hipMemcpyAsync(score_out, score, sizeof(float) * (size_t)T.rows,
                          hipMemcpyDeviceToDevice, st);
  return hipGetLastError();
}

hipError_t launch_adam(float* prop, const float* grad, float* m1, float* m2, float lr,
                       float beta1, float beta2, float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((kParams + 255) / 256)), dim3(256), 0, st, prop,
                     grad, m1, m2, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace lg

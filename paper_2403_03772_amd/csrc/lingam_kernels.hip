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
//   m1 = -2 alpha log2(e) |t|    (the pair constant dithered over the lanes
//                                 between its two FP32 neighbours: one FP32
//                                 rounding of it would bias every sample the
//                                 same way)
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
#include "lingam_device.h"

namespace lg {
namespace {

__global__ __launch_bounds__(1024) void k_setup_schedule(const JobDev* __restrict__ jobs,
                                                         int njobs, int32_t* spre) {
  __shared__ int32_t sh[1024];
  for (int kind = 0; kind < kNumSetupKinds; ++kind)
    block_scan(
        njobs, [&](int j) { return setup_count(jobs[j].n_pad, jobs[j].d, kind); },
        spre + (int64_t)kind * (njobs + 1), sh);
}

// Exclusive prefix sums of one value per lane over the first `count` lanes
// of a wave (inclusive in the return value's last lane).
__device__ inline int32_t wave_excl_scan(int32_t v, int32_t& total) {
  const int lane = threadIdx.x & 63;
  int32_t incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  total = __shfl(incl, 63);
  return incl - v;
}

// Schedule of a batch of at most 64 jobs: in every wave of the block lane j
// plans job j (the same plan in each wave, so no barrier is needed), wave 0
// stores the plans, and the waves share out the kinds' prefix sums.  Same
// arithmetic as the block path below.
__device__ void step_schedule_wave(const JobDev* __restrict__ jobs, int njobs, int t,
                                   int num_cu, Tune tu, JobStep* __restrict__ js,
                                   int32_t* __restrict__ pre) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  JobStep s{};
  long long mine = 0, mine_c = 0;
  if (lane < njobs) {
    const JobDev& J = jobs[lane];
    s = job_step_base(J.d, t, J.prop ? J.K : 0, J.min_m, J.record != nullptr);
    if (s.m >= 2 && !s.fp64) mine = 2LL * s.ntiles;
    if (s.learned) mine_c = 2LL * s.nct;
  }
  long long items = mine, items_c = mine_c;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    items += __shfl_xor(items, off);
    items_c += __shfl_xor(items_c, off);
  }
  if (lane < njobs) {
    const JobDev& J = jobs[lane];
    job_split(s, J.n_pad, items, num_cu, tu);
    job_split_cand(s, J.n_pad, items_c, num_cu, tu, J.tie_on != 0);
    if (wave == 0) js[lane] = s;
  }
  for (int kind = wave; kind < kNumKinds; kind += nwaves) {
    const int32_t c = lane < njobs ? kind_count(s, kind) : 0;
    int32_t total;
    const int32_t ex = wave_excl_scan(c, total);
    int32_t* out = pre + (int64_t)kind * (njobs + 1);
    if (lane < njobs) out[lane] = ex;
    if (lane == 0) out[njobs] = total;
  }
}

__global__ __launch_bounds__(1024) void k_step_schedule(const JobDev* __restrict__ jobs,
                                                        int njobs, int t, int num_cu, Tune tu,
                                                        JobStep* __restrict__ js,
                                                        int32_t* __restrict__ pre) {
  if (njobs <= 64) {  // uniform over the block
    step_schedule_wave(jobs, njobs, t, num_cu, tu, js, pre);
    return;
  }
  __shared__ long long items, items_c;
  const int tid = threadIdx.x;
  if (tid == 0) items = items_c = 0;
  __syncthreads();
  long long mine = 0, mine_c = 0;
  for (int j = tid; j < njobs; j += 1024) {
    const JobDev& J = jobs[j];
    const JobStep s = job_step_base(J.d, t, J.prop ? J.K : 0, J.min_m, J.record != nullptr);
    js[j] = s;
    if (s.m >= 2 && !s.fp64) mine += 2LL * s.ntiles;
    if (s.learned) mine_c += 2LL * s.nct;
  }
  if (mine) atomicAdd(reinterpret_cast<unsigned long long*>(&items), (unsigned long long)mine);
  if (mine_c)
    atomicAdd(reinterpret_cast<unsigned long long*>(&items_c), (unsigned long long)mine_c);
  __syncthreads();
  for (int j = tid; j < njobs; j += 1024) {
    JobStep s = js[j];
    const JobDev& J = jobs[j];
    job_split(s, J.n_pad, items, num_cu, tu);
    job_split_cand(s, J.n_pad, items_c, num_cu, tu, J.tie_on != 0);
    js[j] = s;
  }
  __syncthreads();
  // the kinds' prefix sums are independent: one wave per kind, 64 jobs at a
  // time, no block barriers (a block-wide scan per kind took ~50 us for a few
  // hundred jobs)
  const int lane = tid & 63;
  for (int kind = tid >> 6; kind < kNumKinds; kind += 16) {
    int32_t* out = pre + (int64_t)kind * (njobs + 1);
    int32_t run = 0;
    for (int j0 = 0; j0 < njobs; j0 += 64) {
      const int j = j0 + lane;
      const int32_t c = j < njobs ? kind_count(js[j], kind) : 0;
      int32_t total;
      const int32_t ex = wave_excl_scan(c, total);
      if (j < njobs) out[j] = run + ex;
      run += total;
    }
    if (lane == 0) out[njobs] = run;
  }
}

// After the learned decisions: gate off the full step of every job whose
// learned pass chose, and recompute the prefix sums of the gated kinds.  The
// splits are left as planned, so no count exceeds the host's grid.
__global__ __launch_bounds__(1024) void k_gate_schedule(const JobDev* __restrict__ jobs,
                                                        int njobs, JobStep* __restrict__ js,
                                                        int32_t* __restrict__ pre) {
  if (njobs <= 64) {  // one wave, no barriers
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    JobStep s{};
    if (lane < njobs) {
      s = js[lane];
      s.gate = s.learned && jobs[lane].ctrl->full == 0;
      js[lane] = s;
    }
    for (int kind = 0; kind < kNumKinds; ++kind) {
      if (!gated_kind(kind)) continue;
      const int32_t c = lane < njobs ? kind_count(s, kind) : 0;
      int32_t total;
      const int32_t ex = wave_excl_scan(c, total);
      int32_t* out = pre + (int64_t)kind * (njobs + 1);
      if (lane < njobs) out[lane] = ex;
      if (lane == 0) out[njobs] = total;
    }
    return;
  }
  __shared__ int32_t sh[1024];
  for (int j = threadIdx.x; j < njobs; j += 1024) {
    JobStep s = js[j];
    s.gate = s.learned && jobs[j].ctrl->full == 0;
    js[j] = s;
  }
  __syncthreads();
  for (int kind = 0; kind < kNumKinds; ++kind)
    if (gated_kind(kind))
      block_scan(
          njobs, [&](int j) { return kind_count(js[j], kind); },
          pre + (int64_t)kind * (njobs + 1), sh);
}

struct JobPack {
  JobDev j[kJobsPerLaunch];
};

__global__ void k_set_jobs(JobDev* table, int first, JobPack pack, int count) {
  const int k = threadIdx.x;
  if (k < count) table[first + k] = pack.j[k];
}

// ---------------------------------------------------------------------------
// set-up kernels
// ---------------------------------------------------------------------------

// Per job: identity active list, zero control block, the trivial order of d = 1.
__global__ __launch_bounds__(256) void k_init(const JobDev* __restrict__ jobs) {
  const JobDev& J = jobs[blockIdx.x];
  for (int v = threadIdx.x; v < J.d; v += 256) {
    J.act[v] = v;
    if (J.cmark) J.cmark[v] = 0;
    if (J.steplog) J.steplog[v] = 0;
  }
  if (threadIdx.x < (int)(sizeof(Ctrl) / sizeof(int32_t)))
    reinterpret_cast<int32_t*>(J.ctrl)[threadIdx.x] = 0;
  if (threadIdx.x == 0 && J.d == 1) J.order[0] = 0;
}

// Samples (optionally gathered through `rows`) -> Zd[v][s] (FP64, exact), zero
// padding for s >= n and for row v == d; row d of the FP32 copy Z is zeroed
// too.  Non-finite input or a row index outside [0, n_src) is reported.
__global__ __launch_bounds__(256) void k_ingest(const JobDev* __restrict__ jobs, int njobs,
                                                const int32_t* __restrict__ spre) {
  __shared__ float tile[64][65];
  int j, lb;
  if (!locate(spre, njobs, blockIdx.x, j, lb)) return;
  const JobDev& J = jobs[j];
  if (!J.X) return;  // data rows pre-filled by the caller of the engine
  const int gx = J.n_pad / 64;
  const int s0 = (lb % gx) * 64, v0 = (lb / gx) * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  bool bad = false, badrow = false;
  for (int i = 0; i < 16; ++i) {
    const int sl = ty * 16 + i, s = s0 + sl, v = v0 + tx;
    float val = 0.f;
    if (s < J.n && v < J.d) {
      int64_t row = s;
      if (J.rows) {
        row = J.rows[s];
        if (row < 0 || row >= J.n_src) {
          badrow = true;
          row = -1;
        }
      }
      if (row >= 0) {
        val = J.X[row * J.ldx + v];
        bad |= !isfinite(val);
      }
    }
    tile[sl][tx] = val;
  }
  __syncthreads();
  for (int i = 0; i < 16; ++i) {
    const int vl = ty * 16 + i, v = v0 + vl, s = s0 + tx;
    if (v <= J.d && s < J.n_pad) {
      J.zd[(int64_t)v * J.ldz + s] = (double)tile[tx][vl];
      if (v == J.d) J.z[(int64_t)v * J.ldz + s] = 0.f;
    }
  }
  if (bad) set_status(J.ctrl, kStDegenerate);
  if (badrow) set_status(J.ctrl, kStInvalid);
}

// Population mean and std (two passes, FP64) of each variable.
__global__ __launch_bounds__(256) void k_moments(const JobDev* __restrict__ jobs, int njobs,
                                                 const int32_t* __restrict__ spre) {
  __shared__ double sh[256];
  int j, v;
  if (!locate(spre, njobs, blockIdx.x, j, v)) return;
  const JobDev& J = jobs[j];
  const int n = J.n;
  const double* z = J.zd + (int64_t)v * J.ldz;
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
      set_status(J.ctrl, kStDegenerate);
      sd = 1.0;
    }
    J.mu[v] = m;
    J.sig[v] = sd;
  }
}

typedef double double4_t __attribute__((ext_vector_type(4)));

// Correlation matrix rho = C / (n sigma_i sigma_j), C = sum_s (x_i - mu_i)(x_j - mu_j),
// on FP64 MFMA (v_mfma_f64_16x16x4f64).  One workgroup per 32 x 32 tile of the
// upper triangle, four waves each owning a 16 x 16 block; samples staged
// through LDS in chunks of 32, centred on the way in.
__global__ __launch_bounds__(256) void k_gram(const JobDev* __restrict__ jobs, int njobs,
                                              const int32_t* __restrict__ spre) {
  constexpr int KC = 32;
  __shared__ double As[KC][33];
  __shared__ double Bs[KC][33];
  int jb, tile;
  if (!locate(spre + (int64_t)kSGram * (njobs + 1), njobs, blockIdx.x, jb, tile)) return;
  const JobDev& J = jobs[jb];
  const int d = J.d, n = J.n, n_pad = J.n_pad;
  const int64_t ldz = J.ldz, ldr = d;
  const int nb = cdiv(d, 32);
  int bi, bj;
  decode_tile(tile, nb, bi, bj);
  const int I0 = bi * 32, J0 = bj * 32;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  // loader mapping: 32 variables x 32 samples, 4 consecutive samples per thread
  const int lv = tid >> 3, ls = (tid & 7) * 4;
  const int va = I0 + lv, vb = J0 + lv;
  const double* za = J.zd + (int64_t)(va < d ? va : d) * ldz;  // row d is all zeros
  const double* zb = J.zd + (int64_t)(vb < d ? vb : d) * ldz;
  const double mua = va < d ? J.mu[va] : 0.0, mub = vb < d ? J.mu[vb] : 0.0;
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
    const int jj = J0 + wj * 16 + (lane & 15);
    if (i < d && jj < d && (bi != bj || i <= jj)) {
      double v = acc[r] / ((double)n * J.sig[i] * J.sig[jj]);
      if (i == jj) v = 1.0;
      else if (!(fabs(v) < 1.0 - kCollinear)) degenerate = true;
      J.rho[(int64_t)i * ldr + jj] = v;
      J.rho[(int64_t)jj * ldr + i] = v;
    }
  }
  if (degenerate) set_status(J.ctrl, kStDegenerate);
}

// z = (x - mu) / sigma in place in FP64, its FP32 copy, and the marginal
// entropy H(z) of every variable (FP64).
__global__ __launch_bounds__(256) void k_standardize(const JobDev* __restrict__ jobs, int njobs,
                                                     const int32_t* __restrict__ spre) {
  __shared__ double sh[5 * 4];
  int j, v;
  if (!locate(spre, njobs, blockIdx.x, j, v)) return;
  const JobDev& J = jobs[j];
  double* zd = J.zd + (int64_t)v * J.ldz;
  float* zf = J.z + (int64_t)v * J.ldz;
  const double m = J.mu[v], is = 1.0 / J.sig[v];
  const int n = J.n;
  MomAcc ma;
  for (int k = threadIdx.x; k < J.n_pad; k += 256) {
    if (k < n) {
      const double z = (zd[k] - m) * is;
      zd[k] = z;
      zf[k] = (float)z;
      ma.add(z);
    } else {
      zf[k] = 0.f;
    }
  }
  double acc[5];
  ma.sums(acc);
  block_sum_5(acc, sh);
  if (threadIdx.x == 0) store_moments(J, v, acc, n);
}

// ---------------------------------------------------------------------------
// the step kernels
// ---------------------------------------------------------------------------

template <int W>
__global__ __launch_bounds__(64 * W) void k_pair(const JobDev* __restrict__ jobs, int njobs,
                                                 const JobStep* __restrict__ js,
                                                 const int32_t* __restrict__ pre, int G) {
  pair_tiles<kModeAll, false, W>(jobs, njobs, js, pre, G);
}

// The same kernel for gated launches (learned form): a bounded grid walks the
// step's items.
template <int W>
__global__ __launch_bounds__(64 * W) void k_pair_loop(const JobDev* __restrict__ jobs,
                                                         int njobs,
                                                         const JobStep* __restrict__ js,
                                                         const int32_t* __restrict__ pre,
                                                         int G) {
  pair_tiles<kModeAll, true, W>(jobs, njobs, js, pre, G);
}

// Sum the sample splits (FP64, fixed order), form both residual entropies and
// the likelihood ratio of every pair, write R by position (antisymmetric).
// The S1 sums carry an offset of nsplit * 64 * kS1Start + 0.5 n_pad.
__global__ __launch_bounds__(256) void k_combine(const JobDev* __restrict__ jobs, int njobs,
                                                 const JobStep* __restrict__ js,
                                                 const int32_t* __restrict__ pre) {
  for_blocks(pre, njobs, [&](int jb, int lb) {
  const JobDev& J = jobs[jb];
  const JobStep S = js[jb];
  const int gid = lb * 256 + threadIdx.x;
  if (gid >= S.ntiles * 64) return;
  const int tile = gid >> 6, wave = (gid >> 4) & 3, q = gid & 15;
  int bi, bj;
  decode_tile_st(tile, S.nblk, bi, bj);
  const int wi = wave >> 1, wj = wave & 1;
  const int m = S.m;
  const int pi = bi * kTileVars + wi * kWaveVars + (q >> 2);
  const int pj = bj * kTileVars + wj * kWaveVars + (q & 3);
  if (!(pi < m && pj < m && pi < pj)) return;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int sp = 0; sp < S.nsplit; ++sp) {
    const double* src = J.part + (((int64_t)sp * S.ntiles + tile) * 4 + wave) * 64 + q * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) s[c] += src[c];
  }
  const double s1_bias = (double)S.nsplit * 64.0 * (double)kS1Start + 0.5 * (double)J.n_pad;
  const double inv_n = 1.0 / (double)J.n;
  const int si = J.act[pi], sj = J.act[pj];
  double r = J.rho[(int64_t)si * J.d + sj];
  const double lim = 1.0 - kCollinear;
  r = r > lim ? lim : (r < -lim ? -lim : r);
  const double al = 1.0 / sqrt(1.0 - r * r);
  const double h_ij = entropy_from_moments(kLn2 * (s[0] + s1_bias) * inv_n, al * s[1] * inv_n);
  const double h_ji = entropy_from_moments(kLn2 * (s[2] + s1_bias) * inv_n, al * s[3] * inv_n);
  const double Rv = (J.hm[sj] + h_ij) - (J.hm[si] + h_ji);
  J.rmat[(int64_t)pi * J.d + pj] = Rv;
  J.rmat[(int64_t)pj * J.d + pi] = -Rv;
  });
}

// The same measure entirely in FP64 from the FP64 residuals, for steps with few
// active variables.  One wave per unordered pair (both directions), lanes over
// samples, FP64 wave reduction; writes R(i,j) and R(j,i) = -R(i,j).
__global__ __launch_bounds__(256) void k_pair64(const JobDev* __restrict__ jobs, int njobs,
                                                const JobStep* __restrict__ js,
                                                const int32_t* __restrict__ pre) {
  for_blocks(pre, njobs, [&](int jb, int lb) {
  const JobDev& J = jobs[jb];
  const int m = js[jb].m;
  const int lane = threadIdx.x & 63;
  const int pair = lb * 4 + (threadIdx.x >> 6);
  const int npairs = m * (m - 1) / 2;
  if (pair >= npairs) return;
  int pi = 0, rem = pair;
  while (rem >= m - 1 - pi) {
    rem -= m - 1 - pi;
    ++pi;
  }
  const int pj = pi + 1 + rem;
  const double Rv = pair_measure64(J, pi, pj, lane);
  if (lane == 0) {
    J.rmat[(int64_t)pi * J.d + pj] = Rv;
    J.rmat[(int64_t)pj * J.d + pi] = -Rv;
  }
  });
}

// k_p = sum_{q != p} min(0, R(p, q))^2, one wave per row; mvec[p] = -k_p.
__global__ __launch_bounds__(256) void k_rowk(const JobDev* __restrict__ jobs, int njobs,
                                              const JobStep* __restrict__ js,
                                              const int32_t* __restrict__ pre) {
  for_blocks(pre, njobs, [&](int jb, int lb) {
  const JobDev& J = jobs[jb];
  const int m = js[jb].m;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lb * 4 + wave;
  if (p >= m) return;
  const double* row = J.rmat + (int64_t)p * J.d;
  double k = 0.0;
  for (int q = lane; q < m; q += 64) {
    if (q == p) continue;
    const double x = row[q];
    const double ng = x < 0.0 ? x : 0.0;
    k += ng * ng;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) k += __shfl_xor(k, off);
  if (lane == 0) J.mvec[p] = -k;
  });
}

// Argmax with tie-break on the original id, teacher forcing, per-step outputs,
// swap-remove of the chosen variable.  One workgroup of 1024 threads per job.
__global__ __launch_bounds__(1024) void k_select(const JobDev* __restrict__ jobs, int njobs,
                                                 const JobStep* __restrict__ js,
                                                 const int32_t* __restrict__ pre, int t) {
  __shared__ Best sh[1024];
  __shared__ int forced_pos, ntie;
  for_blocks(pre, njobs, [&](int jb, int) {
  const JobDev& J = jobs[jb];
  const int m = js[jb].m, d = J.d;
  int32_t* act = J.act;
  const int tid = threadIdx.x;
  if (tid == 0) forced_pos = -1;
  __syncthreads();
  Best b{-INFINITY, 0x7fffffff, -1, -INFINITY};
  const bool force = t < J.forced_len;
  const int want = force ? J.forced[t] : -1;
  for (int p = tid; p < m; p += 1024) {
    double v = J.mvec[p];
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
      if (tid == 0) set_status(J.ctrl, kStInvalid);
    } else {
      pos = forced_pos;
    }
  }
  if (J.measures) {
    double* row = J.measures + (int64_t)t * d;
    for (int v = tid; v < d; v += 1024) row[v] = NAN;
    __syncthreads();
    for (int p = tid; p < m; p += 1024) row[act[p]] = J.mvec[p];
  }
  // near-tie: every position whose k is within tie_limit of the best goes to
  // the FP64 decision (FP32 steps, not forced, at most kMaxTie of them)
  if (tid == 0) ntie = 0;
  __syncthreads();
  const bool refine = J.tie_on && !force && !js[jb].fp64 && best.pos >= 0;
  if (refine) {
    const double lim = tie_limit(-best.v);
    for (int p = tid; p < m; p += 1024) {
      const double k = -J.mvec[p];
      if (k <= lim) {
        const int w = atomicAdd(&ntie, 1);
        if (w < kMaxTie) J.tie[w] = p;
      }
    }
  }
  __syncthreads();
  const bool defer = refine && ntie >= 2 && ntie <= kMaxTie;
  if (tid == 0 && refine && ntie > kMaxTie) J.ctrl->n_tie_overflow += 1;
  if (tid == 0) {
    const bool audit = js[jb].learned && J.audit_every > 0 && t % J.audit_every == 0;
    if (J.gaps) J.gaps[t] = best.v - best.v2;
    if (defer) {  // k_tie commits
      J.ctrl->ntie = ntie;
      J.ctrl->tie_t = t;
      J.ctrl->tie_done = 0;
      for (int r = 0; r < kMaxTie; ++r) J.ctrl->tie_row_done[r] = 0;
      J.ctrl->tie_audit = audit ? 1 : 0;
    } else {
      const int slot = act[pos];
      if (audit && slot == J.ctrl->learned_slot) J.ctrl->n_audit_agree += 1;
      J.order[t] = slot;
      J.ctrl->exo_slot = slot;
      J.ctrl->exo_pos = pos;
      act[pos] = act[m - 1];
      if (m == 2) J.order[t + 1] = act[0];
    }
  }
  __syncthreads();  // the next job's item reuses the shared arrays
  });
}

// The FP64 decision of deferred near-ties.  Pairs (r, j) for every listed
// position r and every active position j of every job that deferred at this
// step: both residual directions over all samples in FP64 from the FP64
// residuals (the arithmetic of k_pair64), one wave per pair, R(r, r) = 0.
// The pairs of all such jobs form one list, jobs in index order, that the
// waves of the grid take in turn, so a step where a few jobs of a large batch
// tie still spreads over the whole device.  Every workgroup rebuilds the list
// boundaries from the jobs' control blocks (256 jobs at a time); those fields
// are written by the selection before this launch and only read here.  Each
// listed row counts its finished pairs (ctrl->tie_row_done); the wave that
// finishes a row's last pair sums that row's k in FP64 (columns in a fixed
// order) into the slot after the rows, and the wave that finishes the job's
// last row (ctrl->tie_done) takes the largest -k with ties to the smaller
// original id and commits it as the full selection commits.
__device__ void tie_row_k(const JobDev& J, int m, int r, int lane) {
  const double* row = J.tie_r + (int64_t)r * J.d;
  double k = 0.0;
  for (int q = lane; q < m; q += 64) {
    const double x = row[q];
    const double ng = x < 0.0 ? x : 0.0;
    k += ng * ng;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) k += __shfl_xor(k, off);
  if (lane == 0) J.tie_r[(int64_t)kMaxTie * J.d + r] = k;
}

__device__ void tie_commit(const JobDev& J, int m, int nt, int t) {
  Ctrl* C = J.ctrl;
  int32_t* act = J.act;
  const double* sk = J.tie_r + (int64_t)kMaxTie * J.d;
  int bi = 0;
  for (int r = 1; r < nt; ++r) {
    const double a = sk[r], b = sk[bi];
    if (a < b || (a == b && act[J.tie[r]] < act[J.tie[bi]])) bi = r;
  }
  const int pos = J.tie[bi], slot = act[pos];
  if (C->tie_audit && slot == C->learned_slot) C->n_audit_agree += 1;
  J.order[t] = slot;
  C->exo_slot = slot;
  C->exo_pos = pos;
  act[pos] = act[m - 1];
  C->n_ties += 1;
  C->n_tie_rows += nt;
}

__global__ __launch_bounds__(256) void k_tie(const JobDev* __restrict__ jobs, int njobs,
                                             const JobStep* __restrict__ js, int t) {
  __shared__ int64_t spre[256];  // inclusive prefix of pair counts, this chunk of jobs
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t gw = (int64_t)blockIdx.x * 4 + (tid >> 6), nw = (int64_t)gridDim.x * 4;
  int64_t base = 0;  // pairs of the jobs before this chunk
  for (int j0 = 0; j0 < njobs; j0 += 256) {
    const int jc = j0 + tid;
    int64_t c = 0;
    if (jc < njobs) {
      const Ctrl* C = jobs[jc].ctrl;
      const int nt = C->ntie;
      if (C->tie_t == t && nt >= 2) c = (int64_t)nt * js[jc].m;
    }
    spre[tid] = c;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int64_t v = tid >= off ? spre[tid - off] : 0;
      __syncthreads();
      spre[tid] += v;
      __syncthreads();
    }
    const int64_t total = spre[255];
    // this wave's pairs: list indices w = gw (mod nw) inside [base, base + total)
    int64_t w = base + ((gw - base % nw) % nw + nw) % nw;
    for (; w < base + total; w += nw) {
      const int64_t loc = w - base;
      int lo = 0, hi = 255;  // first job of the chunk whose prefix exceeds loc
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (spre[mid] > loc) hi = mid;
        else lo = mid + 1;
      }
      const JobDev& J = jobs[j0 + lo];
      Ctrl* C = J.ctrl;
      const int m = js[j0 + lo].m;
      const int64_t q = loc - (lo ? spre[lo - 1] : 0);
      const int r = (int)(q / m), pj = (int)(q - (int64_t)r * m);
      const int pi = J.tie[r];
      double* out = J.tie_r + (int64_t)r * J.d + pj;
      const double Rv = pi == pj ? 0.0 : pair_measure64(J, pi, pj, lane);
      if (lane == 0) *out = Rv;
      __threadfence();
      int done = 0;
      if (lane == 0) done = atomicAdd(&C->tie_row_done[r], 1) + 1;
      done = __shfl(done, 0);
      if (done != m) continue;  // wave-uniform
      __threadfence();
      tie_row_k(J, m, r, lane);  // the row's last pair: its k
      __threadfence();
      int rows = 0;
      if (lane == 0) rows = atomicAdd(&C->tie_done, 1) + 1;
      rows = __shfl(rows, 0);
      if (rows == C->ntie && lane == 0) {  // the job's last row: the decision
        __threadfence();
        tie_commit(J, m, rows, t);
      }
    }
    base += total;
    __syncthreads();  // spre is rewritten for the next chunk
  }
}

// Remove the chosen variable e from every remaining variable p and keep p
// standardized: z_p <- (z_p - rho_pe z_e) / sqrt(1 - rho_pe^2) in FP64, refresh
// the FP32 copy, recompute H(z_p) in FP64, update row p of the correlation
// matrix.  One workgroup per remaining variable.
__global__ __launch_bounds__(256) void k_resid(const JobDev* __restrict__ jobs, int njobs,
                                               const JobStep* __restrict__ js,
                                               const int32_t* __restrict__ pre) {
  __shared__ double sh[5 * 4];
  int jb, p;
  if (!locate(pre, njobs, blockIdx.x, jb, p)) return;
  const JobDev& J = jobs[jb];
  const int m_after = js[jb].m - 1;
  const int64_t ldz = J.ldz, ldr = J.d;
  const int sp = J.act[p], se = J.ctrl->exo_slot;
  const double* rho_e = J.rho + (int64_t)se * ldr;
  const double r = rho_e[sp];
  double om = 1.0 - r * r;
  if (!(fabs(r) < 1.0 - kCollinear)) {
    if (threadIdx.x == 0) set_status(J.ctrl, kStDegenerate);
    om = 1.0;
  }
  const double al = 1.0 / sqrt(om);
  double* zp = J.zd + (int64_t)sp * ldz;
  const double* ze = J.zd + (int64_t)se * ldz;
  float* zf = J.z + (int64_t)sp * ldz;
  const int n = J.n;
  MomAcc ma;
  // four samples per thread in flight: all loads are issued before the stores
  // (the rows of p and e are distinct), the samples are added in index order
  constexpr int kU = 4;
  const int n_pad = J.n_pad;
  for (int k0 = threadIdx.x; k0 < n_pad; k0 += 256 * kU) {
    double a[kU], b[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + u * 256;
      a[u] = k < n_pad ? zp[k] : 0.0;
      b[u] = k < n_pad ? ze[k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int k = k0 + u * 256;
      if (k < n_pad) {
        const double z = al * (a[u] - r * b[u]);  // padded samples stay 0
        zp[k] = z;
        zf[k] = (float)z;
        if (k < n) ma.add(z);
      }
    }
  }
  double acc[5];
  ma.sums(acc);
  block_sum_5(acc, sh);
  if (threadIdx.x == 0) store_moments(J, sp, acc, n);
  double* rho_p = J.rho + (int64_t)sp * ldr;
  for (int q = threadIdx.x; q < m_after; q += 256) {
    if (q == p) continue;
    const int sq = J.act[q];
    const double rq = rho_e[sq];
    double oq = 1.0 - rq * rq;
    if (!(fabs(rq) < 1.0 - kCollinear)) oq = 1.0;  // flagged by q's own workgroup
    rho_p[sq] = (rho_p[sq] - r * rq) / sqrt(om * oq);
  }
}

__global__ void k_gather_status(const JobDev* __restrict__ jobs, int njobs, int32_t* dst) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < njobs) dst[j] = jobs[j].ctrl->status;
}

// X row-major [n x ldx] -> Zd[v][s] (FP64) for the VAR series: zero padding
// for s >= n and row d.
// Sample s of the output is row s of X, or row rows[s] when a row map is given
// (indices are checked before the launch).
__global__ __launch_bounds__(256) void k_transpose_f64(const float* __restrict__ X, int64_t ldx,
                                                       const int32_t* __restrict__ rows,
                                                       int n, int d, int n_pad,
                                                       double* __restrict__ Zd, int64_t ldz,
                                                       Ctrl* ctrl) {
  __shared__ float tile[64][65];
  const int s0 = blockIdx.x * 64, v0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  bool bad = false;
  for (int i = 0; i < 16; ++i) {
    const int sl = ty * 16 + i, s = s0 + sl, v = v0 + tx;
    float val = 0.f;
    if (s < n && v < d) {
      val = X[(int64_t)(rows ? rows[s] : s) * ldx + v];
      bad |= !isfinite(val);
    }
    tile[sl][tx] = val;
  }
  __syncthreads();
  for (int i = 0; i < 16; ++i) {
    const int vl = ty * 16 + i, v = v0 + vl, s = s0 + tx;
    if (v <= d && s < n_pad) Zd[(int64_t)v * ldz + s] = (double)tile[tx][vl];
  }
  if (bad) set_status(ctrl, kStDegenerate);
}

// ---------------------------------------------------------------------------
// VarLiNGAM: least-squares VAR(k) with intercept, residuals, B0
// ---------------------------------------------------------------------------

// Column q of the lagged design over rows r = 0 .. N-1 (time t = r + lags):
// q = 0: the intercept (ones); q = 1 + (tau - 1) d + v: x_v(t - tau);
// q = 1 + lags d + v: the response x_v(t).  Xd is variable-major [d][ldx].
__device__ inline const double* design_col(int q, const double* Xd, int64_t ldx, int d, int lags,
                                           const double* ones) {
  if (q == 0) return ones;
  const int p = 1 + lags * d;
  if (q < p) {
    const int tau = (q - 1) / d + 1, v = (q - 1) - (tau - 1) * d;
    return Xd + (int64_t)v * ldx + (lags - tau);
  }
  return Xd + (int64_t)(q - p) * ldx + lags;
}

__global__ void k_fill(double* p, int n, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// W = D^T D for the lagged design D (N rows, q = 1 + lags d + d columns), FP64
// MFMA, upper 32 x 32 tiles mirrored.  Same tiling as k_gram, uncentred.
__global__ __launch_bounds__(256) void k_gram_design(const double* __restrict__ Xd, int64_t ldx,
                                                     const double* __restrict__ ones, int d,
                                                     int lags, int N, int q, int nb,
                                                     double* __restrict__ W, int64_t ldw) {
  constexpr int KC = 32;
  __shared__ double As[KC][33];
  __shared__ double Bs[KC][33];
  int bi, bj;
  decode_tile(blockIdx.x, nb, bi, bj);
  const int I0 = bi * 32, J0 = bj * 32;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int lv = tid >> 3, ls = (tid & 7) * 4;
  const int va = I0 + lv, vb = J0 + lv;
  const double* za = design_col(va < q ? va : 0, Xd, ldx, d, lags, ones);
  const double* zb = design_col(vb < q ? vb : 0, Xd, ldx, d, lags, ones);
  double4_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int s0 = 0; s0 < N; s0 += KC) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int s = s0 + ls + u;
      As[ls + u][lv] = (s < N && va < q) ? za[s] : 0.0;
      Bs[ls + u][lv] = (s < N && vb < q) ? zb[s] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const double a = As[kk * 4 + (lane >> 4)][wi * 16 + (lane & 15)];
      const double b = Bs[kk * 4 + (lane >> 4)][wj * 16 + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = I0 + wi * 16 + 4 * r + (lane >> 4);
    const int j = J0 + wj * 16 + (lane & 15);
    if (i < q && j < q && (bi != bj || i <= j)) {
      W[(int64_t)i * ldw + j] = acc[r];
      W[(int64_t)j * ldw + i] = acc[r];
    }
  }
}

// Residuals e_v(r) = x_v(r + lags) - sum_q D[r][q] A[q][v] into the ordering's
// FP64 data rows Zd[v][r]; optional FP32 row-major copy; VAR matrices M.
__global__ __launch_bounds__(64) void k_var_resid(const double* __restrict__ Xd, int64_t ldx,
                                                  int d,
                                                  int lags, int N, const double* __restrict__ W,
                                                  int64_t ldw, double* __restrict__ Zd,
                                                  int64_t ldz, float* resid_out,
                                                  double* M_out) {
  const int r = blockIdx.x;
  const int v = blockIdx.y * 64 + threadIdx.x;
  if (v >= d) return;
  const int p = 1 + lags * d;
  const double* A = W + p;  // A[q][v] = W[q][p + v]
  double e = Xd[(int64_t)v * ldx + r + lags] - A[v];  // response minus intercept
  for (int tau = 1; tau <= lags; ++tau) {
    const double* Aq = A + (int64_t)(1 + (tau - 1) * d) * ldw;
    for (int u = 0; u < d; ++u)
      e -= Xd[(int64_t)u * ldx + r + lags - tau] * Aq[(int64_t)u * ldw + v];
  }
  Zd[(int64_t)v * ldz + r] = e;
  if (resid_out) resid_out[(int64_t)r * d + v] = (float)e;
  if (M_out && r == 0) {
    // M[tau-1][i][j] = coefficient of x_j(t - tau) in the equation of x_i
    for (int tau = 1; tau <= lags; ++tau)
      for (int j = 0; j < d; ++j)
        M_out[((int64_t)(tau - 1) * d + v) * d + j] = A[(int64_t)(1 + (tau - 1) * d + j) * ldw + v];
  }
}

// Zero the sample padding of Zd rows 0..d-1 and all of row d of Zd and Z.
__global__ void k_zero_pad(double* Zd, float* Z, int64_t ldz, int d, int n, int n_pad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tail = (int64_t)(n_pad - n);
  if (i < (int64_t)d * tail) {
    const int v = (int)(i / tail), r = n + (int)(i - (int64_t)v * tail);
    Zd[(int64_t)v * ldz + r] = 0.0;
  }
  if (i < n_pad) {
    Zd[(int64_t)d * ldz + i] = 0.0;
    Z[(int64_t)d * ldz + i] = 0.f;
  }
}

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

// Status kInvalid unless order is a permutation of 0 .. d-1 (mark starts at 0)
// and every row index rows[0 .. n-1] (if given) lies in [0, n_rows).
__global__ __launch_bounds__(1024) void k_check_perm(const int32_t* __restrict__ order, int d,
                                                     const int32_t* __restrict__ rows, int64_t n,
                                                     int64_t n_rows, int32_t* __restrict__ mark,
                                                     Ctrl* ctrl) {
  for (int i = threadIdx.x; i < d; i += 1024) {
    const int v = order[i];
    if (v < 0 || v >= d || atomicAdd(&mark[v], 1) != 0) set_status(ctrl, kStInvalid);
  }
  if (rows)
    for (int64_t s = threadIdx.x; s < n; s += 1024)
      if (rows[s] < 0 || rows[s] >= n_rows) set_status(ctrl, kStInvalid);
}

// Bootstrap counts of one resample: order_count[i][j] += 1 when x_j precedes
// x_i; edge_count[i][j] += 1 when |B[i][j]| > thr; coef_sum += B (if given).
__global__ void k_boot_accumulate(const int32_t* __restrict__ order,
                                  const double* __restrict__ B, int d, double thr,
                                  int32_t* __restrict__ order_count,
                                  int32_t* __restrict__ edge_count,
                                  double* __restrict__ coef_sum) {
  const int64_t total = (int64_t)d * d;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e / d), b = (int)(e - (int64_t)a * d);  // positions a > b
    if (a > b) {
      const int oa = order[a], ob = order[b];
      if ((unsigned)oa < (unsigned)d && (unsigned)ob < (unsigned)d)  // never write outside
        order_count[(int64_t)oa * d + ob] += 1;
    }
    const double w = B[e];
    if (fabs(w) > thr) edge_count[e] += 1;
    if (coef_sum) coef_sum[e] += w;
  }
}

// Bootstrap probabilities: the counts (and the coefficient sum) divided by the
// number of resamples.
__global__ void k_boot_finalize(const int32_t* __restrict__ order_count,
                                const int32_t* __restrict__ edge_count,
                                const double* __restrict__ coef_sum, int64_t total, double inv,
                                double* __restrict__ order_prob, double* __restrict__ edge_prob,
                                double* __restrict__ coef_mean) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    order_prob[e] = (double)order_count[e] * inv;
    edge_prob[e] = (double)edge_count[e] * inv;
    if (coef_sum) coef_mean[e] = coef_sum[e] * inv;
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side: layouts, schedules, launchers
// ---------------------------------------------------------------------------

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(int64_t n, int64_t d, int num_cu, int K) {
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
  // partial sums: the most splits any policy in range can give a job alone
  // (a batch only ever splits less)
  const Tune worst{kMaxTargetPerCu, kMinMinIters, 4, 4};
  size_t pe = 0;
  for (int64_t t = 0; t + kFp64MaxM < d; ++t) {
    JobStep s = job_step_base((int32_t)d, (int32_t)t);
    job_split(s, (int32_t)L.n_pad, 2LL * s.ntiles, num_cu, worst);
    const size_t need = (size_t)s.ntiles * (size_t)s.nsplit * 256;
    if (need > pe) pe = need;
  }
  L.part_elems = pe;
  L.part = take(sizeof(double) * (pe ? pe : 1));
  L.rmat = take(sizeof(double) * (size_t)d * (size_t)d);
  L.mvec = take(sizeof(double) * (size_t)d);
  L.mom = take(sizeof(double) * 8 * (size_t)d);
  L.tie = take(sizeof(int32_t) * kMaxTie);
  L.tie_r = take(sizeof(double) * kMaxTie * ((size_t)d + 1));
  L.K = K;
  if (K > 0) {
    L.feat = take(sizeof(float) * kFeat * (size_t)d);
    L.score = take(sizeof(float) * (size_t)d);
    L.cand = take(sizeof(int32_t) * kMaxTopK);
    L.cmark = take(sizeof(int32_t) * (size_t)d);
    size_t pc = 0;
    for (int64_t t = 0; t + kFp64MaxM < d; ++t) {
      JobStep s = job_step_base((int32_t)d, (int32_t)t, K, 0, false);
      if (!s.learned) continue;
      job_split(s, (int32_t)L.n_pad, 2LL * s.ntiles, num_cu, worst);
      // either split policy (own split, or the full step's)
      for (const bool own : {true, false}) {
        job_split_cand(s, (int32_t)L.n_pad, 2LL * s.nct, num_cu, worst, own);
        const size_t need = (size_t)s.nct * (size_t)s.nsplit_c * 256;
        if (need > pc) pc = need;
      }
    }
    L.partc_elems = pc;
    L.partc = take(sizeof(double) * (pc ? pc : 1));
    L.rc = take(sizeof(double) * (size_t)K * (size_t)d);
    L.kc = take(sizeof(double) * (size_t)K);
    L.lb = take(sizeof(double) * (size_t)d);
    L.wit = take(sizeof(int32_t) * (size_t)d * kWit);
    L.ext = take(sizeof(int32_t) * kMaxExt);
    L.steplog = take(sizeof(int32_t) * (size_t)d);
    int64_t cap = d / 2 - K;
    cap = cap < kMaxSuspects ? cap : kMaxSuspects;
    L.cap_s = cap > 0 ? (int32_t)(cap / 8 * 8) : 0;
    size_t ps = 0;
    for (int64_t t = 0; t + kFp64MaxM < d && L.cap_s > 0; ++t) {
      JobStep s = job_step_base((int32_t)d, (int32_t)t, K, 0, false);
      if (!s.learned) continue;
      job_split(s, (int32_t)L.n_pad, 2LL * s.ntiles, num_cu, worst);
      const int32_t cs = suspect_cap(s.m, s.k, L.cap_s);
      const size_t tiles = (size_t)cdiv(cs, kTileVars) * s.nblk;
      // the full step's split (extension columns; suspect rows without the
      // FP64 tie resolution), and the suspect pass's own: with T tiles it
      // takes at most ceil(target / 2T) splits, so T * splits <= T + target / 2
      const size_t own = tiles + (size_t)num_cu * worst.target_per_cu / 2 + 1;
      const size_t need = (tiles * (size_t)s.nsplit > own ? tiles * (size_t)s.nsplit : own) * 256;
      if (need > ps) ps = need;
    }
    L.parts_elems = ps;
    L.cand2 = take(sizeof(int32_t) * (size_t)(L.cap_s > 0 ? L.cap_s : 1));
    L.parts = take(sizeof(double) * (ps ? ps : 1));
    L.rc2 = take(sizeof(double) * (size_t)(L.cap_s > 0 ? L.cap_s : 1) * (size_t)d);
    L.kc2 = take(sizeof(double) * (size_t)(L.cap_s > 0 ? L.cap_s : 1));
  }
  L.total = off;
  return L;
}

size_t sched_bytes(int njobs) {
  return align256(sizeof(JobStep) * (size_t)njobs) +
         align256(sizeof(int32_t) * (size_t)kNumKinds * (size_t)(njobs + 1)) +
         align256(sizeof(int32_t) * (size_t)kNumSetupKinds * (size_t)(njobs + 1));
}

SchedDev sched_at(char* base, int njobs) {
  SchedDev s;
  s.js = reinterpret_cast<JobStep*>(base);
  char* p = base + align256(sizeof(JobStep) * (size_t)njobs);
  s.pre = reinterpret_cast<int32_t*>(p);
  p += align256(sizeof(int32_t) * (size_t)kNumKinds * (size_t)(njobs + 1));
  s.spre = reinterpret_cast<int32_t*>(p);
  return s;
}

static inline const int32_t* pre_of(SchedDev sc, int njobs, int kind) {
  return sc.pre + (int64_t)kind * (njobs + 1);
}
static inline const int32_t* spre_of(SchedDev sc, int njobs, int kind) {
  return sc.spre + (int64_t)kind * (njobs + 1);
}

hipError_t launch_set_jobs(JobDev* table, int first, const JobDev* host_jobs, int count,
                           hipStream_t st) {
  JobPack pack{};
  for (int k = 0; k < count && k < kJobsPerLaunch; ++k) pack.j[k] = host_jobs[k];
  hipLaunchKernelGGL(k_set_jobs, dim3(1), dim3(kJobsPerLaunch), 0, st, table, first, pack, count);
  return hipGetLastError();
}

hipError_t launch_setup_schedule(const JobDev* jobs, int njobs, SchedDev sc, hipStream_t st) {
  hipLaunchKernelGGL(k_setup_schedule, dim3(1), dim3(1024), 0, st, jobs, njobs, sc.spre);
  return hipGetLastError();
}

hipError_t launch_init(const JobDev* jobs, int njobs, hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3((unsigned)njobs), dim3(256), 0, st, jobs);
  return hipGetLastError();
}

hipError_t launch_ingest(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ingest, dim3((unsigned)grid), dim3(256), 0, st, jobs, njobs,
                     spre_of(sc, njobs, kSIngest));
  return hipGetLastError();
}

hipError_t launch_moments(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_moments, dim3((unsigned)grid), dim3(256), 0, st, jobs, njobs,
                     spre_of(sc, njobs, kSCols));
  return hipGetLastError();
}

hipError_t launch_gram(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gram, dim3((unsigned)grid), dim3(256), 0, st, jobs, njobs, sc.spre);
  return hipGetLastError();
}

hipError_t launch_standardize(const JobDev* jobs, int njobs, SchedDev sc, int grid,
                              hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_standardize, dim3((unsigned)grid), dim3(256), 0, st, jobs, njobs,
                     spre_of(sc, njobs, kSCols));
  return hipGetLastError();
}

hipError_t launch_step_schedule(const JobDev* jobs, int njobs, int t, int num_cu, Tune tu,
                                SchedDev sc, hipStream_t st) {
  hipLaunchKernelGGL(k_step_schedule, dim3(1), dim3(1024), 0, st, jobs, njobs, t, num_cu, tu,
                     sc.js, sc.pre);
  return hipGetLastError();
}

hipError_t launch_gate_schedule(const JobDev* jobs, int njobs, SchedDev sc, hipStream_t st) {
  hipLaunchKernelGGL(k_gate_schedule, dim3(1), dim3(1024), 0, st, jobs, njobs, sc.js, sc.pre);
  return hipGetLastError();
}

template <int W>
static void launch_pair_w(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st,
                          bool loop) {
  if (loop)
    hipLaunchKernelGGL(k_pair_loop<W>, dim3((unsigned)grid), dim3(64 * W), 0, st, jobs, njobs,
                       (const JobStep*)sc.js, pre_of(sc, njobs, kKPair), grid);
  else
    hipLaunchKernelGGL(k_pair<W>, dim3((unsigned)grid), dim3(64 * W), 0, st, jobs, njobs,
                       (const JobStep*)sc.js, pre_of(sc, njobs, kKPair), grid);
}

hipError_t launch_pair(const JobDev* jobs, int njobs, SchedDev sc, int grid, int waves,
                       hipStream_t st, bool loop) {
  if (grid <= 0) return hipSuccess;
  if (waves == 1) launch_pair_w<1>(jobs, njobs, sc, grid, st, loop);
  else if (waves == 2) launch_pair_w<2>(jobs, njobs, sc, grid, st, loop);
  else launch_pair_w<4>(jobs, njobs, sc, grid, st, loop);
  return hipGetLastError();
}

hipError_t launch_tie(const JobDev* jobs, int njobs, SchedDev sc, int t, int num_cu,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_tie, dim3((unsigned)(num_cu * 4)), dim3(256), 0, st, jobs, njobs,
                     (const JobStep*)sc.js, t);
  return hipGetLastError();
}

hipError_t launch_combine(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine, dim3((unsigned)grid), dim3(256), 0, st, jobs, njobs,
                     (const JobStep*)sc.js, pre_of(sc, njobs, kKComb));
  return hipGetLastError();
}

hipError_t launch_pair64(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair64, dim3((unsigned)grid), dim3(256), 0, st, jobs, njobs,
                     (const JobStep*)sc.js, pre_of(sc, njobs, kKP64));
  return hipGetLastError();
}

hipError_t launch_rowk(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rowk, dim3((unsigned)grid), dim3(256), 0, st, jobs, njobs,
                     (const JobStep*)sc.js, pre_of(sc, njobs, kKRowk));
  return hipGetLastError();
}

hipError_t launch_select(const JobDev* jobs, int njobs, int t, SchedDev sc, int grid,
                         hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_select, dim3((unsigned)grid), dim3(1024), 0, st, jobs, njobs,
                     (const JobStep*)sc.js, pre_of(sc, njobs, kKSel), t);
  return hipGetLastError();
}

hipError_t launch_resid(const JobDev* jobs, int njobs, SchedDev sc, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_resid, dim3((unsigned)grid), dim3(256), 0, st, jobs, njobs,
                     (const JobStep*)sc.js, pre_of(sc, njobs, kKRes));
  return hipGetLastError();
}

hipError_t launch_gather_status(const JobDev* jobs, int njobs, int32_t* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_status, dim3((unsigned)((njobs + 255) / 256)), dim3(256), 0, st,
                     jobs, njobs, dst);
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

VarLayout make_var_layout(int64_t T, int64_t d, int lags, int num_cu) {
  VarLayout V{};
  V.T = T;
  V.d = d;
  V.lags = lags;
  V.N = T - lags;
  V.p = 1 + (int64_t)lags * d;
  V.q = V.p + d;
  V.ord = make_layout(V.N, d, num_cu);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  V.ldx = (T + 63) / 64 * 64;
  V.xd = take(sizeof(double) * (size_t)(d + 1) * (size_t)V.ldx);
  V.ones = take(sizeof(double) * (size_t)V.N);
  V.w = take(sizeof(double) * (size_t)V.q * (size_t)V.q);
  V.rho0 = take(sizeof(double) * (size_t)d * (size_t)d);
  V.scr = take(sizeof(double) * (size_t)d * (size_t)d);
  V.y = take(sizeof(double) * (size_t)d * (size_t)d);
  V.tol = take(sizeof(double));
  V.linv = take(sizeof(double) * (size_t)V.p * (size_t)V.p);
  V.tmp = take(sizeof(double) * (size_t)V.p * (size_t)d);
  V.total = off;
  return V;
}

hipError_t launch_var_fit(const VarLayout& V, char* ws, char* job, const float* X,
                          int64_t ldx_in, float* resid_out, double* M_out, hipStream_t st) {
  const Layout& L = V.ord;
  Ctrl* ctrl = at<Ctrl>(job, L.ctrl);
  double* Xd = at<double>(ws, V.xd);
  double* ones = at<double>(ws, V.ones);
  double* W = at<double>(ws, V.w);
  // series -> variable-major FP64 (padding beyond T is zero)
  dim3 g1((unsigned)(V.ldx / 64), (unsigned)((V.d + 1 + 63) / 64));
  hipLaunchKernelGGL(k_transpose_f64, g1, dim3(256), 0, st, X, ldx_in, (const int32_t*)nullptr,
                     (int)V.T, (int)V.d,
                     (int)V.ldx, Xd, V.ldx, ctrl);
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((V.N + 255) / 256)), dim3(256), 0, st, ones,
                     (int)V.N, 1.0);
  const int nb = (int)((V.q + 31) / 32);
  hipLaunchKernelGGL(k_gram_design, dim3((unsigned)(nb * (nb + 1) / 2)), dim3(256), 0, st, Xd,
                     V.ldx, ones, (int)V.d, V.lags, (int)V.N, (int)V.q, nb, W, V.q);
  LG_HIP(launch_cholesky(W, V.q, (int)V.p, at<double>(ws, V.tol), ctrl, st));
  // coefficients (L L^T)^-1 C = X^T (X C), X = L^-1, C = W[0:p, p:q]
  double* Xi = at<double>(ws, V.linv);
  double* T = at<double>(ws, V.tmp);
  LG_HIP(launch_tri_inverse(W, V.q, (int)V.p, Xi, V.p, st));
  LG_HIP(launch_trmm((int)V.p, (int)V.d, Xi, V.p, false, W + V.p, V.q, T, V.d, st));
  LG_HIP(launch_trmm((int)V.p, (int)V.d, Xi, V.p, true, T, V.d, W + V.p, V.q, st));
  dim3 g2((unsigned)V.N, (unsigned)((V.d + 63) / 64));
  hipLaunchKernelGGL(k_var_resid, g2, dim3(64), 0, st, Xd, V.ldx, (int)V.d, V.lags, (int)V.N,
                     W, V.q, at<double>(job, L.zd), L.ldz, resid_out, M_out);
  const int64_t zn = (L.d * (L.n_pad - L.n) > L.n_pad) ? L.d * (L.n_pad - L.n) : L.n_pad;
  hipLaunchKernelGGL(k_zero_pad, dim3((unsigned)((zn + 255) / 256)), dim3(256), 0, st,
                     at<double>(job, L.zd), at<float>(job, L.z), L.ldz, (int)L.d, (int)L.n,
                     (int)L.n_pad);
  return hipGetLastError();
}

hipError_t launch_save_rho(const VarLayout& V, char* ws, char* job, hipStream_t st) {
  return hipMemcpyAsync(ws + V.rho0, job + V.ord.rho, sizeof(double) * (size_t)(V.d * V.d),
                        hipMemcpyDeviceToDevice, st);
}

// B0: least squares of every residual on its order predecessors, from the
// residual covariance diag(sig) rho0 diag(sig) permuted into the order.
hipError_t launch_b0(const VarLayout& V, char* ws, char* job, const int32_t* order, double* B0,
                     hipStream_t st) {
  double* S = at<double>(ws, V.scr);
  LG_HIP(launch_perm_scale(at<double>(ws, V.rho0), V.d, at<double>(job, V.ord.sig), order,
                           (int)V.d, S, st));
  LG_HIP(launch_cholesky(S, V.d, (int)V.d, at<double>(ws, V.tol), at<Ctrl>(job, V.ord.ctrl), st));
  return launch_tri_adjacency(S, V.d, (int)V.d, order, B0, at<double>(ws, V.y), st);
}

// ---------------------------------------------------------------------------
// least-squares adjacency from a causal order
// ---------------------------------------------------------------------------

AdjLayout make_adj_layout(int64_t n, int64_t d) {
  AdjLayout A{};
  A.n = n;
  A.d = d;
  A.ldx = (n + 63) / 64 * 64;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  A.ctrl = take(sizeof(Ctrl));
  A.mark = take(sizeof(int32_t) * (size_t)d);
  A.tol = take(sizeof(double));
  A.mu = take(sizeof(double) * (size_t)d);
  A.xd = take(sizeof(double) * (size_t)(d + 1) * (size_t)A.ldx);
  A.s = take(sizeof(double) * (size_t)d * (size_t)d);
  A.y = take(sizeof(double) * (size_t)d * (size_t)d);
  A.total = off;
  return A;
}

hipError_t launch_adj_check(const AdjLayout& A, char* ws, const int32_t* order,
                            const int32_t* rows, int64_t n_rows, hipStream_t st) {
  Ctrl* ctrl = at<Ctrl>(ws, A.ctrl);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, st, &ctrl->status);
  const int64_t g = (A.d + 255) / 256;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)(g < 1024 ? g : 1024)), dim3(256), 0, st,
                     at<int32_t>(ws, A.mark), A.d, 0);
  hipLaunchKernelGGL(k_check_perm, dim3(1), dim3(1024), 0, st, order, (int)A.d, rows, A.n,
                     n_rows, at<int32_t>(ws, A.mark), ctrl);
  return hipGetLastError();
}

hipError_t launch_adjacency(const AdjLayout& A, char* ws, const float* X, int64_t ldx,
                            const int32_t* rows, const int32_t* order, double* B,
                            hipStream_t st) {
  Ctrl* ctrl = at<Ctrl>(ws, A.ctrl);
  double* Xd = at<double>(ws, A.xd);
  double* S = at<double>(ws, A.s);
  dim3 g1((unsigned)(A.ldx / 64), (unsigned)((A.d + 1 + 63) / 64));
  hipLaunchKernelGGL(k_transpose_f64, g1, dim3(256), 0, st, X, ldx, rows, (int)A.n, (int)A.d,
                     (int)A.ldx, Xd, A.ldx, ctrl);
  LG_HIP(launch_cov_perm(Xd, A.ldx, (int)A.n, (int)A.d, order, at<double>(ws, A.mu), S, st));
  LG_HIP(launch_cholesky(S, A.d, (int)A.d, at<double>(ws, A.tol), ctrl, st));
  return launch_tri_adjacency(S, A.d, (int)A.d, order, B, at<double>(ws, A.y), st);
}

hipError_t launch_boot_accumulate(const int32_t* order, const double* B, int d, double thr,
                                  int32_t* order_count, int32_t* edge_count, double* coef_sum,
                                  hipStream_t st) {
  const int64_t g = ((int64_t)d * d + 255) / 256;
  hipLaunchKernelGGL(k_boot_accumulate, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, st,
                     order, B, d, thr, order_count, edge_count, coef_sum);
  return hipGetLastError();
}

hipError_t launch_boot_finalize(const int32_t* order_count, const int32_t* edge_count,
                                const double* coef_sum, int d, int32_t n_resamples,
                                double* order_prob, double* edge_prob, double* coef_mean,
                                hipStream_t st) {
  const int64_t total = (int64_t)d * d, g = (total + 255) / 256;
  hipLaunchKernelGGL(k_boot_finalize, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, st,
                     order_count, edge_count, coef_sum, total, 1.0 / (double)n_resamples,
                     order_prob, edge_prob, coef_mean);
  return hipGetLastError();
}

}  // namespace lg

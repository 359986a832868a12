// gfx950 dense FP64 linear algebra of the library.
//
//   blocked Cholesky     A = L L^T by 32-wide panels: the diagonal block is
//                        factored in LDS by one workgroup, the panel below it
//                        is solved row-parallel against that block (rows
//                        staged in LDS), and the trailing lower triangle takes
//                        the rank-32 update on FP64 MFMA (16 x 16 x 4), one
//                        32 x 32 tile per workgroup.
//   adjacency from L     least squares of every variable on the variables
//                        that precede it in a causal order (the second phase
//                        of DirectLiNGAM, Section 1; B0 of VarLiNGAM, Section
//                        3.3).  With the covariance permuted into the order,
//                        S = L L^T, the coefficients of variable o_i on
//                        o_0 .. o_{i-1} solve S_i b = s_i with S_i = L_i L_i^T
//                        (leading i x i blocks) and s_i = L_i l_i (l_i = row i
//                        of L left of the diagonal), so b = L_i^-T l_i.
//                        Stacked over i this is B = I - diag(L) L^-1.
//   triangular inverse   X = L^-1 by 32 x 32 blocks: the diagonal blocks are
//                        inverted in LDS (all at once), then block row I is
//                        X_IJ = -X_II sum_{J <= K < I} L_IK X_KJ for all J < I
//                        in one launch (both products on FP64 MFMA), so the
//                        dependency chain is p / 32 launches long.
//   triangular products  op(X) B for the normal equations of the VAR fit:
//                        (L L^T)^-1 C = X^T (X C).
//   covariance           centred Gram matrix of variable rows, permuted into
//                        a given order, on FP64 MFMA.
//   lagged effects       theta_tau = (I - B0) M_tau of VarLiNGAM (Section
//                        3.3: the model's lagged matrices from the VAR ones).
#include "lingam_device.h"
#include "lingam_linalg.h"

namespace lg {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kNb = 32;  // Cholesky panel width and update tile

// tol = 1e-13 * max_j |A_jj|: pivots at or below it are rounding noise.
__global__ __launch_bounds__(256) void k_chol_tol(const double* __restrict__ A, int64_t lda,
                                                  int p, double* __restrict__ tol) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (int j = threadIdx.x; j < p; j += 256) mx = fmax(mx, fabs(A[(int64_t)j * lda + j]));
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) tol[0] = sh[0] * 1e-13;
}

// Factor the kb x kb diagonal block at (k0, k0) (lower triangle) in LDS.
__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ A, int64_t lda, int k0,
                                                   int kb, const double* __restrict__ tol,
                                                   Ctrl* ctrl) {
  __shared__ double T[kNb][kNb + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < kNb * kNb; e += 256) {
    const int i = e / kNb, j = e - i * kNb;
    T[i][j] = (i < kb && j <= i) ? A[(int64_t)(k0 + i) * lda + k0 + j] : 0.0;
  }
  __syncthreads();
  const double tl = tol[0];
  for (int j = 0; j < kb; ++j) {
    if (tid == 0) {
      double a = T[j][j];
      if (!(a > tl) || !isfinite(a)) {
        set_status(ctrl, kStDegenerate);
        a = 1.0;
      }
      T[j][j] = sqrt(a);
    }
    __syncthreads();
    if (tid > j && tid < kb) T[tid][j] /= T[j][j];
    __syncthreads();
    const int w = kb - j - 1;
    for (int e = tid; e < w * w; e += 256) {
      const int ii = e / w, kk = e - ii * w;
      if (kk <= ii) T[j + 1 + ii][j + 1 + kk] -= T[j + 1 + ii][j] * T[j + 1 + kk][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < kb * kb; e += 256) {
    const int i = e / kb, j = e - i * kb;
    if (j <= i) A[(int64_t)(k0 + i) * lda + k0 + j] = T[i][j];
  }
}

// Rows i >= r0 = k0 + kb of the panel: A[i, k0:k0+kb] <- A[i, k0:k0+kb] L_kk^-T
// (forward substitution along the row; one thread per row, the rows staged
// in LDS, 64 rows per workgroup).
constexpr int kPanelRows = 64;

__global__ __launch_bounds__(kPanelRows) void k_chol_panel(double* __restrict__ A, int64_t lda,
                                                           int p, int k0, int kb) {
  __shared__ double Lk[kNb][kNb + 1];
  __shared__ double X[kPanelRows][kNb + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < kNb * kNb; e += kPanelRows) {
    const int i = e / kNb, j = e - i * kNb;
    Lk[i][j] = (i < kb && j <= i) ? A[(int64_t)(k0 + i) * lda + k0 + j] : 0.0;
  }
  const int rbase = k0 + kb + blockIdx.x * kPanelRows;
  // coalesced staging: consecutive threads take consecutive columns of a row
  for (int e = tid; e < kPanelRows * kNb; e += kPanelRows) {
    const int r = e / kNb, c = e - r * kNb;
    X[r][c] = (rbase + r < p && c < kb) ? A[(int64_t)(rbase + r) * lda + k0 + c] : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < kb; ++c) {
    double s = X[tid][c];
    for (int t = 0; t < c; ++t) s -= X[tid][t] * Lk[c][t];
    X[tid][c] = s / Lk[c][c];
  }
  __syncthreads();
  for (int e = tid; e < kPanelRows * kNb; e += kPanelRows) {
    const int r = e / kNb, c = e - r * kNb;
    if (rbase + r < p && c < kb) A[(int64_t)(rbase + r) * lda + k0 + c] = X[r][c];
  }
}

// Trailing update of the lower triangle right of the panel:
// A[i][j] -= sum_c A[i][k0 + c] A[j][k0 + c] for r0 <= j <= i < p, r0 = k0 + kb.
// One 32 x 32 tile (I >= J) per workgroup, four waves of 16 x 16 on MFMA.
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ A, int64_t lda, int p,
                                                     int k0, int kb, int nt) {
  __shared__ double As[kNb][kNb + 1];
  __shared__ double Bs[kNb][kNb + 1];
  int bj, bi;
  decode_tile(blockIdx.x, nt, bj, bi);  // bj <= bi: tile (I, J) = (bi, bj) is lower
  const int r0 = k0 + kb;
  const int I0 = r0 + bi * kNb, J0 = r0 + bj * kNb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int lv = tid >> 3, ls = (tid & 7) * 4;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = ls + u;
    As[c][lv] = (c < kb && I0 + lv < p) ? A[(int64_t)(I0 + lv) * lda + k0 + c] : 0.0;
    Bs[c][lv] = (c < kb && J0 + lv < p) ? A[(int64_t)(J0 + lv) * lda + k0 + c] : 0.0;
  }
  __syncthreads();
  double4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < kNb / 4; ++kk) {
    const double a = As[kk * 4 + (lane >> 4)][wi * 16 + (lane & 15)];
    const double b = Bs[kk * 4 + (lane >> 4)][wj * 16 + (lane & 15)];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = I0 + wi * 16 + 4 * r + (lane >> 4);
    const int j = J0 + wj * 16 + (lane & 15);
    if (i < p && j <= i) A[(int64_t)i * lda + j] -= acc[r];
  }
}

// Diagonal 32 x 32 blocks of X = L^-1: X_II = L_II^-1, written in full (zeros
// above the diagonal; past p the block is cut).  One workgroup per block;
// thread j < 32 runs the forward substitution of column j in LDS.
__global__ __launch_bounds__(64) void k_trinv_diag(const double* __restrict__ L, int64_t ldl,
                                                   int p, double* __restrict__ X, int64_t ldx) {
  __shared__ double Ls[kNb][kNb + 1];
  __shared__ double Ds[kNb][kNb + 1];
  const int I0 = blockIdx.x * kNb, kb = min(kNb, p - I0);
  const int tid = threadIdx.x;
  for (int e = tid; e < kNb * kNb; e += 64) {
    const int i = e / kNb, j = e - i * kNb;
    Ls[i][j] = (i < kb && j <= i) ? L[(int64_t)(I0 + i) * ldl + I0 + j] : 0.0;
  }
  __syncthreads();
  if (tid < kb) {
    const int j = tid;
    for (int i = 0; i < kNb; ++i) Ds[i][j] = 0.0;
    Ds[j][j] = 1.0 / Ls[j][j];
    for (int i = j + 1; i < kb; ++i) {
      double s = 0.0;
      for (int t = j; t < i; ++t) s += Ls[i][t] * Ds[t][j];
      Ds[i][j] = -s / Ls[i][i];
    }
  }
  __syncthreads();
  for (int e = tid; e < kb * kb; e += 64) {
    const int i = e / kb, j = e - i * kb;
    X[(int64_t)(I0 + i) * ldx + I0 + j] = Ds[i][j];
  }
}

// Block row I of X = L^-1 left of the diagonal: X_IJ = -X_II sum_{J <= K < I}
// L_IK X_KJ for every J < I (one workgroup each), both products on FP64 MFMA.
// Blocks K < I and J < I are full (only the last block row can be cut by p).
__global__ __launch_bounds__(256) void k_trinv_row(const double* __restrict__ L, int64_t ldl,
                                                   int p, int I, double* __restrict__ X,
                                                   int64_t ldx) {
  __shared__ double As[kNb][kNb + 1];
  __shared__ double Bs[kNb][kNb + 1];
  const int J = blockIdx.x;
  const int I0 = I * kNb, J0 = J * kNb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int lv = tid >> 3, ls = (tid & 7) * 4;
  const bool row_ok = I0 + lv < p;
  double4_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int K = J; K < I; ++K) {
    const int K0 = K * kNb;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      As[ls + u][lv] = row_ok ? L[(int64_t)(I0 + lv) * ldl + K0 + ls + u] : 0.0;  // L_IK[lv][k]
      Bs[lv][ls + u] = X[(int64_t)(K0 + lv) * ldx + J0 + ls + u];                // X_KJ[k][j]
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kNb / 4; ++kk) {
      const double a = As[kk * 4 + (lane >> 4)][wi * 16 + (lane & 15)];
      const double b = Bs[kk * 4 + (lane >> 4)][wj * 16 + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
  }
  __syncthreads();
  // T = acc becomes the right operand; X_II the left one
#pragma unroll
  for (int r = 0; r < 4; ++r) Bs[wi * 16 + 4 * r + (lane >> 4)][wj * 16 + (lane & 15)] = acc[r];
#pragma unroll
  for (int u = 0; u < 4; ++u)
    As[ls + u][lv] = (row_ok && I0 + ls + u < p) ? X[(int64_t)(I0 + lv) * ldx + I0 + ls + u] : 0.0;
  __syncthreads();
  double4_t out = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < kNb / 4; ++kk) {
    const double a = As[kk * 4 + (lane >> 4)][wi * 16 + (lane & 15)];
    const double b = Bs[kk * 4 + (lane >> 4)][wj * 16 + (lane & 15)];
    out = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, out, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = I0 + wi * 16 + 4 * r + (lane >> 4);
    const int j = J0 + wj * 16 + (lane & 15);
    if (i < p) X[(int64_t)i * ldx + j] = -out[r];
  }
}

// B[order[i]][order[k]] = -L_ii X_ik for k < i, 0 otherwise (every entry of B
// written once: order is a permutation).
__global__ void k_adj_scatter(const double* __restrict__ L, int64_t ldl,
                              const double* __restrict__ X, int64_t ldx, int p,
                              const int32_t* __restrict__ order, double* __restrict__ B) {
  const int64_t total = (int64_t)p * p;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / p), k = (int)(e - (int64_t)i * p);
    const double v = k < i ? -L[(int64_t)i * ldl + i] * X[(int64_t)i * ldx + k] : 0.0;
    B[(int64_t)order[i] * p + order[k]] = v;
  }
}

// C = op(A) B for a lower-triangular M x M A (op = A or A^T), B: M x N,
// 32 x 32 output tiles on FP64 MFMA, visiting only the K blocks where op(A)'s
// row block is nonzero.  C must not alias B.
__global__ __launch_bounds__(256) void k_trmm(int M, int N, const double* __restrict__ A,
                                              int64_t lda, int trans, const double* __restrict__ B,
                                              int64_t ldb, double* __restrict__ C, int64_t ldc) {
  __shared__ double As[kNb][kNb + 1];
  __shared__ double Bs[kNb][kNb + 1];
  const int I0 = blockIdx.y * kNb, J0 = blockIdx.x * kNb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int lv = tid >> 3, ls = (tid & 7) * 4;
  const int kbeg = trans ? I0 : 0;
  const int kend = trans ? M : min(M, I0 + kNb);
  double4_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = kbeg; k0 < kend; k0 += kNb) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (!trans) {  // op(A)[i][k] = A[i][k]: lv = i, ls + u = k
        const int i = I0 + lv, k = k0 + ls + u;
        As[ls + u][lv] = (i < M && k < M) ? A[(int64_t)i * lda + k] : 0.0;
      } else {       // op(A)[i][k] = A[k][i]: lv = k, ls + u = i
        const int k = k0 + lv, i = I0 + ls + u;
        As[lv][ls + u] = (i < M && k < M) ? A[(int64_t)k * lda + i] : 0.0;
      }
      const int k = k0 + lv, j = J0 + ls + u;
      Bs[lv][ls + u] = (k < M && j < N) ? B[(int64_t)k * ldb + j] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kNb / 4; ++kk) {
      const double a = As[kk * 4 + (lane >> 4)][wi * 16 + (lane & 15)];
      const double b = Bs[kk * 4 + (lane >> 4)][wj * 16 + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = I0 + wi * 16 + 4 * r + (lane >> 4);
    const int j = J0 + wj * 16 + (lane & 15);
    if (i < M && j < N) C[(int64_t)i * ldc + j] = acc[r];
  }
}

// S[a][b] = sig[o_a] sig[o_b] rho[o_a][o_b]: a correlation matrix scaled to a
// covariance and permuted into the order o.
__global__ void k_perm_scale(const double* __restrict__ rho, int64_t ldr,
                             const double* __restrict__ sig, const int32_t* __restrict__ order,
                             int d, double* __restrict__ S) {
  const int64_t total = (int64_t)d * d;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e / d), b = (int)(e - (int64_t)a * d);
    const int oa = order[a], ob = order[b];
    S[e] = sig[oa] * sig[ob] * rho[(int64_t)oa * ldr + ob];
  }
}

// mu[v] = mean of row v of Xd over its first n entries (one workgroup per row).
__global__ __launch_bounds__(256) void k_row_mean(const double* __restrict__ Xd, int64_t ldx, int n,
                                                  double* __restrict__ mu) {
  __shared__ double sh[256];
  const double* x = Xd + (int64_t)blockIdx.x * ldx;
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += x[k];
  s = block_sum_256(s, sh);
  if (threadIdx.x == 0) mu[blockIdx.x] = s / (double)n;
}

// S[a][b] = sum_s (x_{o_a}(s) - mu_{o_a}) (x_{o_b}(s) - mu_{o_b}) on FP64 MFMA,
// upper 32 x 32 tiles computed and mirrored.
__global__ __launch_bounds__(256) void k_cov_perm(const double* __restrict__ Xd, int64_t ldx,
                                                  int n, int d,
                                                  const int32_t* __restrict__ order,
                                                  const double* __restrict__ mu, int nb,
                                                  double* __restrict__ S) {
  constexpr int KC = 32;
  __shared__ double As[KC][33];
  __shared__ double Bs[KC][33];
  int bi, bj;
  decode_tile(blockIdx.x, nb, bi, bj);
  const int I0 = bi * 32, J0 = bj * 32;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int lv = tid >> 3, ls = (tid & 7) * 4;
  const int va = I0 + lv < d ? order[I0 + lv] : -1;
  const int vb = J0 + lv < d ? order[J0 + lv] : -1;
  const double* za = Xd + (int64_t)(va < 0 ? 0 : va) * ldx;
  const double* zb = Xd + (int64_t)(vb < 0 ? 0 : vb) * ldx;
  const double ma = va < 0 ? 0.0 : mu[va], mb = vb < 0 ? 0.0 : mu[vb];
  double4_t acc = {0.0, 0.0, 0.0, 0.0};
  for (int s0 = 0; s0 < n; s0 += KC) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int s = s0 + ls + u;
      As[ls + u][lv] = (s < n && va >= 0) ? za[s] - ma : 0.0;
      Bs[ls + u][lv] = (s < n && vb >= 0) ? zb[s] - mb : 0.0;
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
    if (i < d && j < d && (bi != bj || i <= j)) {
      S[(int64_t)i * d + j] = acc[r];
      S[(int64_t)j * d + i] = acc[r];
    }
  }
}

// theta[t][i][j] = M[t][i][j] - sum_k B0[i][k] M[t][k][j] (16 x 16 tiles, LDS).
__global__ __launch_bounds__(256) void k_lagged(const double* __restrict__ M,
                                                const double* __restrict__ B0, int d,
                                                double* __restrict__ theta) {
  __shared__ double Bt[16][17];
  __shared__ double Mt[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  const double* Mk = M + (int64_t)blockIdx.z * d * d;
  double s = 0.0;
  for (int k0 = 0; k0 < d; k0 += 16) {
    Bt[ty][tx] = (i < d && k0 + tx < d) ? B0[(int64_t)i * d + k0 + tx] : 0.0;
    Mt[ty][tx] = (k0 + ty < d && j < d) ? Mk[(int64_t)(k0 + ty) * d + j] : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) s += Bt[ty][k] * Mt[k][tx];
    __syncthreads();
  }
  if (i < d && j < d) theta[(int64_t)blockIdx.z * d * d + (int64_t)i * d + j] = Mk[(int64_t)i * d + j] - s;
}

// ---------------------------------------------------------------------------
// adaptive-lasso pruning of the adjacency
// ---------------------------------------------------------------------------

// Xd[v][s] = X[row(s)][v] in FP64 (row(s) = rows[s] or s); padding 0.
__global__ __launch_bounds__(256) void k_gather_f64(const float* __restrict__ X, int64_t ldx,
                                                    const int32_t* __restrict__ rows, int n,
                                                    int d, int n_pad, double* __restrict__ Xd,
                                                    int64_t ldz, Ctrl* ctrl) {
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
    if (v < d && s < n_pad) Xd[(int64_t)v * ldz + s] = (double)tile[tx][vl];
  }
  if (bad) set_status(ctrl, kStDegenerate);
}

// sd[a] = sqrt(S[a][a] / n); R = S scaled to unit diagonal; L = R (to be
// factored).  A zero variance sets the status.
__global__ void k_corr(const double* __restrict__ S, int d, int n, double* __restrict__ sd,
                       double* __restrict__ R, double* __restrict__ L, Ctrl* ctrl) {
  const int64_t total = (int64_t)d * d;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e / d), b = (int)(e - (int64_t)a * d);
    const double saa = S[(int64_t)a * d + a], sbb = S[(int64_t)b * d + b];
    if (!(saa > 0.0) || !(sbb > 0.0)) {
      set_status(ctrl, kStDegenerate);
      R[e] = L[e] = (a == b) ? 1.0 : 0.0;
    } else {
      const double r = S[e] / sqrt(saa * sbb);
      R[e] = L[e] = r;
    }
    if (a == b) sd[a] = sqrt(fmax(saa, 0.0) / (double)n);
  }
}

__global__ void k_zero_f64(double* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

struct LarsShared {
  double M[kLassoMaxActive][kLassoMaxActive + 1];  // inverse of G on the active set
  double g[kLassoMaxActive], v[kLassoMaxActive], wv[kLassoMaxActive];
  double sgn[kLassoMaxActive];
  int idx[kLassoMaxActive];
  int best_idx[kLassoMaxActive];
  double rv[256];
  int ri[256];
  double sv;
  int si;
};

// Block arg-min of (value, index), ties to the smaller index; index -1 = none.
__device__ inline void block_argmin(double v, int i, LarsShared& S, double& ov, int& oi) {
  const int tid = threadIdx.x;
  S.rv[tid] = v;
  S.ri[tid] = i;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) {
      const double a = S.rv[tid], b = S.rv[tid + off];
      const int ia = S.ri[tid], ib = S.ri[tid + off];
      if (ib >= 0 && (ia < 0 || b < a || (b == a && ib < ia))) {
        S.rv[tid] = b;
        S.ri[tid] = ib;
      }
    }
    __syncthreads();
  }
  ov = S.rv[0];
  oi = S.ri[0];
  __syncthreads();
}

__device__ inline double block_sum(double v, LarsShared& S) {
  const int tid = threadIdx.x;
  S.rv[tid] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) S.rv[tid] += S.rv[tid + off];
    __syncthreads();
  }
  const double r = S.rv[0];
  __syncthreads();
  return r;
}

// One workgroup per target position t >= 1 (predictors: positions 0 .. t-1).
// Adaptive weights w_k = |b_k| from the least-squares row of B = I -
// diag(L) L^-1 on the correlation matrix; the lasso path of the weighted
// standardized predictors by least angle regression with the lasso
// modification (covariance form, G_jk = n w_j w_k R_jk, c_k = n w_k R_kt),
// at most max_active active; the breakpoint of least BIC
// n log(2 pi s2) + RSS / s2 + log(n) df, s2 = n L_tt^2 / (n - t - 1); the
// kept predictors refitted by least squares (standardized, then rescaled).
// The path state (correlations, coefficients, directions, flags) lives in
// st[t][4][d]; the inverse of G on the active set in LDS, updated by the
// Schur complement on a join and the rank-1 downdate on a leave.
__global__ __launch_bounds__(256) void k_lars(const double* __restrict__ R,
                                              const double* __restrict__ L,
                                              const double* __restrict__ Y,
                                              const double* __restrict__ sd,
                                              const int32_t* __restrict__ order, int d, int n,
                                              int cap, double* __restrict__ st,
                                              double* __restrict__ B, Ctrl* ctrl) {
  __shared__ LarsShared S;
  const int t = blockIdx.x + 1;
  const int p = t;
  const int tid = threadIdx.x;
  const double nn = (double)n;
  double* corr = st + (int64_t)t * 4 * d;
  double* beta = corr + d;
  double* av = beta + d;
  double* flag = av + d;
  const double Ltt = L[(int64_t)t * d + t];
  const double* Yt = Y + (int64_t)t * d;
  const double* Rt = R + (int64_t)t * d;  // row t = column t (symmetric)
  auto wgt = [&](int k) { return fabs(Ltt * Yt[k]); };
  auto cval = [&](int k) { return nn * wgt(k) * Rt[k]; };
  double cmax = 0.0;
  for (int k = tid; k < p; k += 256) {
    const double c = cval(k);
    corr[k] = c;
    beta[k] = 0.0;
    flag[k] = 0.0;
    cmax = fmax(cmax, fabs(c));
  }
  // max |c| through the arg-min of its negation
  double mv;
  int mi;
  block_argmin(-cmax, tid, S, mv, mi);
  const double tiny = 1e-14 * fmax(1.0, -mv);
  const double s2 = nn * Ltt * Ltt / (double)(n - p - 1);
  const double logterm = nn * log(2.0 * 3.14159265358979323846 * s2);
  const double lnn = log(nn);
  double best = logterm + nn / s2;  // beta = 0: RSS = n, df = 0
  int best_na = 0;
  int na = 0;
  bool joined = true;
  const int cap_a = cap < p ? cap : p;
  const int max_iter = 8 * kLassoMaxActive + 16;  // bound on the loop (never reached in practice)
  for (int iter = 0; iter < max_iter; ++iter) {
    if (joined) {
      if (na == p) break;
      // inactive predictor of largest |corr| (ties to the smaller position)
      double bv = INFINITY;
      int bi = -1;
      for (int k = tid; k < p; k += 256)
        if (flag[k] == 0.0) {
          const double v = -fabs(corr[k]);
          if (v < bv) {
            bv = v;
            bi = k;
          }
        }
      double jv;
      int j;
      block_argmin(bv, bi, S, jv, j);
      if (j < 0 || -jv <= tiny) break;
      // Schur complement: append j to the inverse of G on the active set
      const double wj = wgt(j);
      const double* Rj = R + (int64_t)j * d;
      if (tid < na) S.g[tid] = nn * wgt(S.idx[tid]) * wj * Rj[S.idx[tid]];
      __syncthreads();
      if (tid < na) {
        double acc = 0.0;
        for (int q = 0; q < na; ++q) acc += S.M[tid][q] * S.g[q];
        S.v[tid] = acc;
      }
      __syncthreads();
      if (tid == 0) {
        double gv = 0.0;
        for (int q = 0; q < na; ++q) gv += S.g[q] * S.v[q];
        S.sv = nn * wj * wj * Rj[j] - gv;
      }
      __syncthreads();
      const double sch = S.sv;
      if (!(sch > 1e-12 * nn * wj * wj)) break;  // the new predictor is (nearly) collinear
      for (int e = tid; e < na * na; e += 256) {
        const int r = e / na, q = e - r * na;
        S.M[r][q] += S.v[r] * S.v[q] / sch;
      }
      if (tid < na) {
        S.M[tid][na] = -S.v[tid] / sch;
        S.M[na][tid] = -S.v[tid] / sch;
      }
      if (tid == 0) {
        S.M[na][na] = 1.0 / sch;
        S.idx[na] = j;
        flag[j] = 1.0;
      }
      __syncthreads();
      ++na;
    }
    // equiangular direction on the active set
    if (tid < na) S.sgn[tid] = corr[S.idx[tid]] >= 0.0 ? 1.0 : -1.0;
    __syncthreads();
    if (tid < na) {
      double acc = 0.0;
      for (int q = 0; q < na; ++q) acc += S.M[tid][q] * S.sgn[q];
      S.v[tid] = acc;
    }
    __syncthreads();
    if (tid == 0) {
      double sx = 0.0, cm = 0.0;
      for (int q = 0; q < na; ++q) {
        sx += S.sgn[q] * S.v[q];
        cm = fmax(cm, fabs(corr[S.idx[q]]));
      }
      S.sv = sx;
      S.rv[0] = cm;
    }
    __syncthreads();
    const double AA = 1.0 / sqrt(S.sv);
    const double C = S.rv[0];
    __syncthreads();
    if (tid < na) S.wv[tid] = AA * S.v[tid];
    __syncthreads();
    // a_k = sum_r G(k, idx_r) wv_r, and the first join along the direction
    double gj = INFINITY;
    int kj = -1;
    for (int k = tid; k < p; k += 256) {
      double acc = 0.0;
      for (int r = 0; r < na; ++r) {
        const int ir = S.idx[r];
        acc += nn * wgt(ir) * R[(int64_t)ir * d + k] * S.wv[r];
      }
      acc *= wgt(k);
      av[k] = acc;
      if (flag[k] == 0.0) {
        const double ck = corr[k];
        const double d1 = AA - acc, d2 = AA + acc;
        if (d1 > 0.0) {
          const double g = (C - ck) / d1;
          if (g > 0.0 && g < gj) {
            gj = g;
            kj = k;
          }
        }
        if (d2 > 0.0) {
          const double g = (C + ck) / d2;
          if (g > 0.0 && g < gj) {
            gj = g;
            kj = k;
          }
        }
      }
    }
    double gjoin;
    int jn;
    block_argmin(gj, kj, S, gjoin, jn);
    double gam = C / AA;
    int event = 0;  // 0 end, 1 join, 2 leave
    if (jn >= 0 && gjoin < gam) {
      gam = gjoin;
      event = 1;
    }
    // first active coefficient to reach zero
    double gl = INFINITY;
    int rl = -1;
    if (tid < na && S.wv[tid] != 0.0) {
      const double g = -beta[S.idx[tid]] / S.wv[tid];
      if (g > 0.0) {
        gl = g;
        rl = tid;
      }
    }
    double gleave;
    int lr;
    block_argmin(gl, rl, S, gleave, lr);
    if (lr >= 0 && gleave < gam) {
      gam = gleave;
      event = 2;
    }
    // step
    if (tid < na) beta[S.idx[tid]] += gam * S.wv[tid];
    for (int k = tid; k < p; k += 256) corr[k] -= gam * av[k];
    __syncthreads();
    if (event == 2) {
      const int who = S.idx[lr];
      // rank-1 downdate of the inverse without row / column lr, then compaction
      const double piv = S.M[lr][lr];
      double keep[16];
      const int nb = na - 1;
      int cnt = 0;
      for (int e = tid; e < nb * nb; e += 256, ++cnt) {
        const int r2 = e / nb, q2 = e - r2 * nb;
        const int r = r2 + (r2 >= lr ? 1 : 0), q = q2 + (q2 >= lr ? 1 : 0);
        keep[cnt] = S.M[r][q] - S.M[r][lr] * S.M[lr][q] / piv;
      }
      int idx_keep = tid < nb ? S.idx[tid + (tid >= lr ? 1 : 0)] : 0;
      __syncthreads();
      cnt = 0;
      for (int e = tid; e < nb * nb; e += 256, ++cnt) {
        const int r2 = e / nb, q2 = e - r2 * nb;
        S.M[r2][q2] = keep[cnt];
      }
      if (tid < nb) S.idx[tid] = idx_keep;
      if (tid == 0) {
        beta[who] = 0.0;
        flag[who] = 0.0;
      }
      __syncthreads();
      na = nb;
    }
    // criterion at the new breakpoint: RSS = n - beta'c - beta'corr
    double part = 0.0;
    if (tid < na) {
      const int k = S.idx[tid];
      part = beta[k] * (cval(k) + corr[k]);
    }
    const double bsum = block_sum(part, S);
    const double crit = logterm + (nn - bsum) / s2 + lnn * (double)na;
    if (crit < best) {
      best = crit;
      best_na = na;
      if (tid < na) S.best_idx[tid] = S.idx[tid];
    }
    __syncthreads();
    if (event == 0) break;
    if (event == 1 && na >= cap_a) break;
    joined = event == 1;
  }
  // refit the kept predictors by least squares on the standardized data
  const int ns = best_na;
  if (ns == 0) return;
  for (int e = tid; e < ns * ns; e += 256) {
    const int r = e / ns, q = e - r * ns;
    S.M[r][q] = R[(int64_t)S.best_idx[r] * d + S.best_idx[q]];
  }
  if (tid < ns) S.g[tid] = Rt[S.best_idx[tid]];
  __syncthreads();
  for (int j = 0; j < ns; ++j) {  // Cholesky in LDS, lower triangle
    if (tid == 0) {
      double a = S.M[j][j];
      if (!(a > 1e-13)) {
        set_status(ctrl, kStDegenerate);
        a = 1.0;
      }
      S.M[j][j] = sqrt(a);
    }
    __syncthreads();
    if (tid > j && tid < ns) S.M[tid][j] /= S.M[j][j];
    __syncthreads();
    const int w = ns - j - 1;
    for (int e = tid; e < w * w; e += 256) {
      const int ii = e / w, kk = e - ii * w;
      if (kk <= ii) S.M[j + 1 + ii][j + 1 + kk] -= S.M[j + 1 + ii][j] * S.M[j + 1 + kk][j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int i = 0; i < ns; ++i) {  // forward, then backward substitution
      double acc = S.g[i];
      for (int q = 0; q < i; ++q) acc -= S.M[i][q] * S.g[q];
      S.g[i] = acc / S.M[i][i];
    }
    for (int i = ns - 1; i >= 0; --i) {
      double acc = S.g[i];
      for (int q = i + 1; q < ns; ++q) acc -= S.M[q][i] * S.g[q];
      S.g[i] = acc / S.M[i][i];
    }
  }
  __syncthreads();
  if (tid < ns) {
    const int k = S.best_idx[tid];
    B[(int64_t)order[t] * d + order[k]] = S.g[tid] * sd[t] / sd[k];
  }
}

// A[a][b] = 1 (a == b), -B[o_a][o_b] (a > b), 0 (a < b): I - B in the causal
// order, unit lower triangular (entries of B above that triangle ignored).
__global__ void k_unit_lower(const double* __restrict__ B, const int32_t* __restrict__ order,
                             int d, double* __restrict__ A) {
  const int64_t total = (int64_t)d * d;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e / d), b = (int)(e - (int64_t)a * d);
    A[e] = a == b ? 1.0 : (a > b ? -B[(int64_t)order[a] * d + order[b]] : 0.0);
  }
}

// T[o_a][o_b] = X[a][b] for a >= b, 0 otherwise (every entry written once).
__global__ void k_scatter_lower(const double* __restrict__ X, const int32_t* __restrict__ order,
                                int d, double* __restrict__ T) {
  const int64_t total = (int64_t)d * d;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e / d), b = (int)(e - (int64_t)a * d);
    T[(int64_t)order[a] * d + order[b]] = a >= b ? X[e] : 0.0;
  }
}

unsigned grid_for(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g < 4096 ? (g < 1 ? 1 : g) : 4096);
}

}  // namespace

hipError_t launch_cholesky(double* A, int64_t lda, int p, double* tol, Ctrl* ctrl,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_chol_tol, dim3(1), dim3(256), 0, st, A, lda, p, tol);
  for (int k0 = 0; k0 < p; k0 += kNb) {
    const int kb = p - k0 < kNb ? p - k0 : kNb;
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, st, A, lda, k0, kb, tol, ctrl);
    const int rest = p - k0 - kb;
    if (rest <= 0) break;
    hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)((rest + kPanelRows - 1) / kPanelRows)),
                       dim3(kPanelRows), 0, st, A, lda, p, k0, kb);
    const int nt = (rest + kNb - 1) / kNb;
    hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, st, A,
                       lda, p, k0, kb, nt);
  }
  return hipGetLastError();
}

hipError_t launch_tri_inverse(const double* L, int64_t ldl, int p, double* X, int64_t ldx,
                              hipStream_t st) {
  const int nb = (p + kNb - 1) / kNb;
  hipLaunchKernelGGL(k_trinv_diag, dim3((unsigned)nb), dim3(64), 0, st, L, ldl, p, X, ldx);
  for (int I = 1; I < nb; ++I)
    hipLaunchKernelGGL(k_trinv_row, dim3((unsigned)I), dim3(256), 0, st, L, ldl, p, I, X, ldx);
  return hipGetLastError();
}

hipError_t launch_tri_adjacency(const double* L, int64_t ldl, int p, const int32_t* order,
                                double* B, double* Y, hipStream_t st) {
  LG_HIP(launch_tri_inverse(L, ldl, p, Y, p, st));
  hipLaunchKernelGGL(k_adj_scatter, dim3(grid_for((int64_t)p * p)), dim3(256), 0, st, L, ldl, Y,
                     (int64_t)p, p, order, B);
  return hipGetLastError();
}

hipError_t launch_trmm(int M, int N, const double* A, int64_t lda, bool trans, const double* B,
                       int64_t ldb, double* C, int64_t ldc, hipStream_t st) {
  dim3 g((unsigned)((N + kNb - 1) / kNb), (unsigned)((M + kNb - 1) / kNb));
  hipLaunchKernelGGL(k_trmm, g, dim3(256), 0, st, M, N, A, lda, trans ? 1 : 0, B, ldb, C, ldc);
  return hipGetLastError();
}

hipError_t launch_perm_scale(const double* rho, int64_t ldr, const double* sig,
                             const int32_t* order, int d, double* S, hipStream_t st) {
  hipLaunchKernelGGL(k_perm_scale, dim3(grid_for((int64_t)d * d)), dim3(256), 0, st, rho, ldr,
                     sig, order, d, S);
  return hipGetLastError();
}

hipError_t launch_cov_perm(const double* Xd, int64_t ldx, int n, int d, const int32_t* order,
                           double* mu, double* S, hipStream_t st) {
  hipLaunchKernelGGL(k_row_mean, dim3((unsigned)d), dim3(256), 0, st, Xd, ldx, n, mu);
  const int nb = (d + 31) / 32;
  hipLaunchKernelGGL(k_cov_perm, dim3((unsigned)(nb * (nb + 1) / 2)), dim3(256), 0, st, Xd, ldx,
                     n, d, order, mu, nb, S);
  return hipGetLastError();
}

hipError_t launch_lagged_effects(const double* M, const double* B0, int d, int lags,
                                 double* theta, hipStream_t st) {
  const unsigned g = (unsigned)((d + 15) / 16);
  hipLaunchKernelGGL(k_lagged, dim3(g, g, (unsigned)lags), dim3(256), 0, st, M, B0, d, theta);
  return hipGetLastError();
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

PruneLayout make_prune_layout(int64_t n, int64_t d) {
  PruneLayout A{};
  A.n = n;
  A.d = d;
  A.ldx = (n + 63) / 64 * 64;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  const size_t dd = sizeof(double) * (size_t)d * (size_t)d;
  A.ctrl = take(sizeof(Ctrl));
  A.mark = take(sizeof(int32_t) * (size_t)d);
  A.tol = take(sizeof(double));
  A.mu = take(sizeof(double) * (size_t)d);
  A.sd = take(sizeof(double) * (size_t)d);
  A.xd = take(sizeof(double) * (size_t)d * (size_t)A.ldx);
  A.s = take(dd);
  A.r = take(dd);
  A.l = take(dd);
  A.y = take(dd);
  A.st = take(4 * dd);
  A.total = off;
  return A;
}

hipError_t launch_adjacency_pruned(const PruneLayout& A, char* ws, const float* X, int64_t ldx,
                                   const int32_t* rows, const int32_t* order, int max_active,
                                   double* B, hipStream_t st) {
  Ctrl* ctrl = at<Ctrl>(ws, A.ctrl);
  double* Xd = at<double>(ws, A.xd);
  double* Sm = at<double>(ws, A.s);
  double* Rm = at<double>(ws, A.r);
  double* Lm = at<double>(ws, A.l);
  double* Ym = at<double>(ws, A.y);
  const int d = (int)A.d, n = (int)A.n;
  dim3 g1((unsigned)(A.ldx / 64), (unsigned)((A.d + 63) / 64));
  hipLaunchKernelGGL(k_gather_f64, g1, dim3(256), 0, st, X, ldx, rows, n, d, (int)A.ldx, Xd,
                     A.ldx, ctrl);
  LG_HIP(launch_cov_perm(Xd, A.ldx, n, d, order, at<double>(ws, A.mu), Sm, st));
  const int64_t dd = (int64_t)d * d;
  hipLaunchKernelGGL(k_corr, dim3(grid_for(dd)), dim3(256), 0, st, (const double*)Sm, d, n,
                     at<double>(ws, A.sd), Rm, Lm, ctrl);
  LG_HIP(launch_cholesky(Lm, d, d, at<double>(ws, A.tol), ctrl, st));
  LG_HIP(launch_tri_inverse(Lm, d, d, Ym, d, st));
  hipLaunchKernelGGL(k_zero_f64, dim3(grid_for(dd)), dim3(256), 0, st, B, dd);
  if (d < 2) return hipGetLastError();
  const int cap = max_active < kLassoMaxActive ? max_active : kLassoMaxActive;
  hipLaunchKernelGGL(k_lars, dim3((unsigned)(d - 1)), dim3(256), 0, st, (const double*)Rm,
                     (const double*)Lm, (const double*)Ym, (const double*)at<double>(ws, A.sd),
                     order, d, n, cap, at<double>(ws, A.st), B, ctrl);
  return hipGetLastError();
}

EffectsLayout make_effects_layout(int64_t d) {
  EffectsLayout A{};
  A.d = d;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  A.ctrl = take(sizeof(Ctrl));
  A.mark = take(sizeof(int32_t) * (size_t)d);
  A.a = take(sizeof(double) * (size_t)d * (size_t)d);
  A.x = take(sizeof(double) * (size_t)d * (size_t)d);
  A.total = off;
  return A;
}

hipError_t launch_total_effects(const EffectsLayout& A, char* ws, const double* B,
                                const int32_t* order, double* T, hipStream_t st) {
  const int d = (int)A.d;
  const int64_t dd = (int64_t)d * d;
  double* Am = at<double>(ws, A.a);
  double* Xm = at<double>(ws, A.x);
  hipLaunchKernelGGL(k_unit_lower, dim3(grid_for(dd)), dim3(256), 0, st, B, order, d, Am);
  LG_HIP(launch_tri_inverse(Am, d, d, Xm, d, st));
  hipLaunchKernelGGL(k_scatter_lower, dim3(grid_for(dd)), dim3(256), 0, st, (const double*)Xm,
                     order, d, T);
  return hipGetLastError();
}

}  // namespace lg

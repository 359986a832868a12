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

}  // namespace lg

/*
 * lingam_oracle.c -- plain FP64 CPU oracle for the DirectLiNGAM causal-ordering
 * search (AcceleratedLiNGAM, arXiv 2403.03772).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the yardstick the GPU library is
 * checked against.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  The GPU library never calls it, shares no
 * code, header, table or constant with it, and must never fall back to it.
 *
 * Everything here is deliberately slow and literal:
 *   - FP64 throughout, two-pass means and variances, population (ddof = 0)
 *     moments everywhere,
 *   - the entropy is computed from its definition with log(cosh(u)),
 *   - the "literal" search recomputes the standardisation, both residuals and
 *     all four entropies for every ordered pair, exactly as the causal-ordering
 *     pseudo-implementation (Algorithm 1, Section 2.2) is written,
 *   - the "table" search standardises once per step and evaluates each ordered
 *     residual entropy once (pure memoisation of the same numbers; a test pins
 *     it to the literal search at 1e-12),
 *   - OpenMP parallelises only over candidate variables i (each i writes only
 *     its own k_list entry, so results do not depend on the thread count).
 *
 * Readings of points the paper leaves open (each listed in the design notes):
 *   R1 _diff_mutual_info (named, not defined, in Algorithm 1) is the pairwise
 *      likelihood-ratio measure of Hyvarinen & Smith (2013), which the paper
 *      cites with DirectLiNGAM in Section 1:
 *         diff(i,j) = [H(x_j) + H(r_i^(j)/sd)] - [H(x_i) + H(r_j^(i)/sd)],
 *      positive when i precedes j.
 *   R2 H(.) is the maximum-entropy approximation of differential entropy
 *         H(u) = (1 + log 2pi)/2 - k1 (E log cosh u - gamma)^2
 *                                - k2 (E u exp(-u^2/2))^2
 *      with k1 = 79.047, k2 = 7.4129, gamma = 0.37457, applied to a
 *      unit-variance sample (residuals are divided by their own std first).
 *   R3 _residual(xi, xj) is the least-squares residual xi - (cov/var(xj)) xj,
 *      cov and var with ddof = 0 like np.std in Algorithm 1.
 *   R4 k_list is indexed by position in U (the listing indexes it by value).
 *   R5 np.argmax returns the first maximum; U is kept in ascending original
 *      order, so exact ties go to the smallest original index.
 *   R6 After a variable is chosen, its effect is removed from every remaining
 *      variable by least squares on the raw columns (DirectLiNGAM outer loop,
 *      Section 2.2).
 *   R7 A zero-variance column or a pair with |corr| >= 1 - 1e-12 is reported
 *      as degenerate (status LO_DEGENERATE), never turned into NaN.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* status codes of this oracle (its own; unrelated to the library's) */
#define LO_OK 0
#define LO_INVALID -1
#define LO_DEGENERATE -2
#define LO_NOMEM -3

/* Constants of the entropy approximation (R2). */
static const double LO_K1 = 79.047;
static const double LO_K2 = 7.4129;
static const double LO_GAMMA = 0.37457;

static double lo_hnu(void) { return 0.5 * (1.0 + log(2.0 * M_PI)); }

/* ------------------------------------------------------------------------ */
/* moments (ddof = 0, two-pass)                                              */
/* ------------------------------------------------------------------------ */
static double lo_mean(const double* x, int64_t n) {
  double s = 0.0;
  for (int64_t k = 0; k < n; ++k) s += x[k];
  return s / (double)n;
}

static double lo_var(const double* x, int64_t n) {
  const double mu = lo_mean(x, n);
  double s = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    const double e = x[k] - mu;
    s += e * e;
  }
  return s / (double)n;
}

static double lo_cov(const double* x, const double* y, int64_t n) {
  const double mx = lo_mean(x, n), my = lo_mean(y, n);
  double s = 0.0;
  for (int64_t k = 0; k < n; ++k) s += (x[k] - mx) * (y[k] - my);
  return s / (double)n;
}

/* ------------------------------------------------------------------------ */
/* entropy approximation (R2)                                                */
/* ------------------------------------------------------------------------ */

/* E[log cosh u] and E[u exp(-u^2/2)] of a sample. */
void lo_entropy_moments(const double* u, int64_t n, double* e_logcosh, double* e_gauss) {
  double s1 = 0.0, s2 = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    s1 += log(cosh(u[k]));
    s2 += u[k] * exp(-0.5 * u[k] * u[k]);
  }
  *e_logcosh = s1 / (double)n;
  *e_gauss = s2 / (double)n;
}

/* H(u) for a sample that is already scaled to unit variance. */
double lo_entropy(const double* u, int64_t n) {
  double a, b;
  lo_entropy_moments(u, n, &a, &b);
  return lo_hnu() - LO_K1 * (a - LO_GAMMA) * (a - LO_GAMMA) - LO_K2 * b * b;
}

/* the constants, so tests can pin them against the theory they come from */
void lo_entropy_constants(double* k1, double* k2, double* gamma, double* hnu) {
  *k1 = LO_K1;
  *k2 = LO_K2;
  *gamma = LO_GAMMA;
  *hnu = lo_hnu();
}

/* ------------------------------------------------------------------------ */
/* the pieces of Algorithm 1                                                 */
/* ------------------------------------------------------------------------ */

/* (x - mean(x)) / std(x), ddof = 0.  Returns LO_DEGENERATE on zero std. */
static int lo_standardize(const double* x, int64_t n, double* out) {
  const double mu = lo_mean(x, n);
  const double sd = sqrt(lo_var(x, n));
  if (!(sd > 0.0) || !isfinite(sd)) return LO_DEGENERATE;
  for (int64_t k = 0; k < n; ++k) out[k] = (x[k] - mu) / sd;
  return LO_OK;
}

/* R3: least-squares residual of xi regressed on xj. */
static int lo_residual(const double* xi, const double* xj, int64_t n, double* out) {
  const double vj = lo_var(xj, n);
  if (!(vj > 0.0)) return LO_DEGENERATE;
  const double b = lo_cov(xi, xj, n) / vj;
  for (int64_t k = 0; k < n; ++k) out[k] = xi[k] - b * xj[k];
  return LO_OK;
}

/* H(r / std(r)); `tmp` is scratch of length n. */
static int lo_entropy_of_scaled(const double* r, int64_t n, double* tmp, double* h) {
  const double sd = sqrt(lo_var(r, n));
  if (!(sd > 0.0)) return LO_DEGENERATE;
  for (int64_t k = 0; k < n; ++k) tmp[k] = r[k] / sd;
  *h = lo_entropy(tmp, n);
  return LO_OK;
}

/* R1: difference of mutual informations, from the standardized pair and the
 * two residuals. `tmp` is scratch of length n. */
static int lo_diff_mutual_info(const double* xi_std, const double* xj_std, const double* ri_j,
                               const double* rj_i, int64_t n, double* tmp, double* diff) {
  double h_ri_j, h_rj_i;
  int st = lo_entropy_of_scaled(ri_j, n, tmp, &h_ri_j);
  if (st) return st;
  st = lo_entropy_of_scaled(rj_i, n, tmp, &h_rj_i);
  if (st) return st;
  *diff = (lo_entropy(xj_std, n) + h_ri_j) - (lo_entropy(xi_std, n) + h_rj_i);
  return LO_OK;
}

/* R7 collinearity check on a standardized pair. */
static int lo_check_pair(const double* a, const double* b, int64_t n) {
  const double r = lo_cov(a, b, n) / sqrt(lo_var(a, n) * lo_var(b, n));
  if (!(fabs(r) < 1.0 - 1e-12)) return LO_DEGENERATE;
  return LO_OK;
}

/* The measure for one ordered pair of raw columns, literally as in Algorithm 1.
 * Exported so tests can check antisymmetry and invariances pair by pair. */
int lo_pair_measure(const double* xi, const double* xj, int64_t n, double* diff) {
  if (n < 2) return LO_INVALID;
  double* buf = (double*)malloc(sizeof(double) * 5 * (size_t)n);
  if (!buf) return LO_NOMEM;
  double *xi_std = buf, *xj_std = buf + n, *ri_j = buf + 2 * n, *rj_i = buf + 3 * n,
         *tmp = buf + 4 * n;
  int st = lo_standardize(xi, n, xi_std);
  if (!st) st = lo_standardize(xj, n, xj_std);
  if (!st) st = lo_check_pair(xi_std, xj_std, n);
  if (!st) st = lo_residual(xi_std, xj_std, n, ri_j);
  if (!st) st = lo_residual(xj_std, xi_std, n, rj_i);
  if (!st) st = lo_diff_mutual_info(xi_std, xj_std, ri_j, rj_i, n, tmp, diff);
  free(buf);
  return st;
}

/* ------------------------------------------------------------------------ */
/* one step of the search                                                    */
/* ------------------------------------------------------------------------ */

/* Literal Algorithm 1 on columns Xc[v*n .. v*n+n) for v in U[0..m).
 * Writes k_list[p] = -sum_j min(0, diff(U[p], j))^2 for p in [0, m); rows with
 * want[p] == 0 are skipped (left at NaN) when `want` is non-NULL. */
static int lo_step_literal(const double* Xc, int64_t n, const int32_t* U, int32_t m,
                           const unsigned char* want, double* k_list) {
  int status = LO_OK;
#pragma omp parallel
  {
    double* buf = (double*)malloc(sizeof(double) * 5 * (size_t)n);
    if (!buf) {
#pragma omp atomic write
      status = LO_NOMEM;
    }
#pragma omp for schedule(dynamic, 1)
    for (int32_t p = 0; p < m; ++p) {
      if (!buf) continue;
      if (want && !want[p]) {
        k_list[p] = NAN;
        continue;
      }
      double *xi_std = buf, *xj_std = buf + n, *ri_j = buf + 2 * n, *rj_i = buf + 3 * n,
             *tmp = buf + 4 * n;
      const double* xi = Xc + (int64_t)U[p] * n;
      double k = 0.0;
      int st = LO_OK;
      for (int32_t q = 0; q < m && !st; ++q) {
        if (q == p) continue;
        const double* xj = Xc + (int64_t)U[q] * n;
        double diff = 0.0;
        st = lo_standardize(xi, n, xi_std);
        if (!st) st = lo_standardize(xj, n, xj_std);
        if (!st) st = lo_check_pair(xi_std, xj_std, n);
        if (!st) st = lo_residual(xi_std, xj_std, n, ri_j);
        if (!st) st = lo_residual(xj_std, xi_std, n, rj_i);
        if (!st) st = lo_diff_mutual_info(xi_std, xj_std, ri_j, rj_i, n, tmp, &diff);
        const double neg = diff < 0.0 ? diff : 0.0;
        k += neg * neg;
      }
      if (st) {
#pragma omp atomic write
        status = st;
      }
      k_list[p] = -k;
    }
    free(buf);
  }
  return status;
}

/* The matrix of the likelihood-ratio measure between the active columns:
 * D[p * m + q] = diff(U[p], U[q]) of R1, D[p * m + p] = 0.  Each column is
 * standardized once, each marginal entropy and each ordered residual entropy
 * is computed once, and diff(j, i) is taken as -diff(i, j) (which the formula
 * of R1 gives exactly).  Xc is column-major (column v at Xc + v * n).
 *
 * Pure memoisation of the pair pieces of Algorithm 1: the mean and variance
 * of every standardized column are computed once (lo_mean / lo_var are
 * deterministic, so each is the same number the per-pair calls would give),
 * and the one covariance of a pair serves the collinearity check and both
 * residual slopes (the product (a - ma)(b - mb) is commutative in IEEE
 * arithmetic, so cov(z_i, z_j) and cov(z_j, z_i) are the same number).  The
 * results equal those of lo_check_pair + lo_residual bit for bit. */
int lo_pair_matrix(const double* Xc, int64_t n, const int32_t* U, int32_t m, double* D) {
  double* Z = (double*)malloc(sizeof(double) * (size_t)m * (size_t)n);
  double* Hm = (double*)malloc(sizeof(double) * (size_t)m);
  double* mz = (double*)malloc(sizeof(double) * (size_t)m);
  double* vz = (double*)malloc(sizeof(double) * (size_t)m);
  if (!Z || !Hm || !mz || !vz) {
    free(Z);
    free(Hm);
    free(mz);
    free(vz);
    return LO_NOMEM;
  }
  int status = LO_OK;
#pragma omp parallel for schedule(static)
  for (int32_t p = 0; p < m; ++p) {
    double* zp = Z + (int64_t)p * n;
    int st = lo_standardize(Xc + (int64_t)U[p] * n, n, zp);
    if (st) {
#pragma omp atomic write
      status = st;
    } else {
      Hm[p] = lo_entropy(zp, n);
      mz[p] = lo_mean(zp, n);
      vz[p] = lo_var(zp, n);
    }
  }
  if (status) goto done;
#pragma omp parallel
  {
    double* buf = (double*)malloc(sizeof(double) * 3 * (size_t)n);
#pragma omp for schedule(dynamic, 1)
    for (int32_t p = 0; p < m; ++p) {
      if (!buf) {
#pragma omp atomic write
        status = LO_NOMEM;
        continue;
      }
      double *ri_j = buf, *rj_i = buf + n, *tmp = buf + 2 * n;
      const double* zi = Z + (int64_t)p * n;
      D[(int64_t)p * m + p] = 0.0;
      for (int32_t q = p + 1; q < m; ++q) {
        const double* zj = Z + (int64_t)q * n;
        /* cov(z_i, z_j) exactly as lo_cov computes it */
        double c = 0.0;
        for (int64_t k = 0; k < n; ++k) c += (zi[k] - mz[p]) * (zj[k] - mz[q]);
        c /= (double)n;
        /* R7 (lo_check_pair) */
        if (!(fabs(c / sqrt(vz[p] * vz[q])) < 1.0 - 1e-12)) {
#pragma omp atomic write
          status = LO_DEGENERATE;
          continue;
        }
        /* R3 both ways (lo_residual): slope cov / var of the regressor */
        const double bij = c / vz[q], bji = c / vz[p];
        for (int64_t k = 0; k < n; ++k) {
          ri_j[k] = zi[k] - bij * zj[k];
          rj_i[k] = zj[k] - bji * zi[k];
        }
        double h1 = 0.0, h2 = 0.0;
        int st = lo_entropy_of_scaled(ri_j, n, tmp, &h1);
        if (!st) st = lo_entropy_of_scaled(rj_i, n, tmp, &h2);
        if (st) {
#pragma omp atomic write
          status = st;
          continue;
        }
        const double diff = (Hm[q] + h1) - (Hm[p] + h2);
        D[(int64_t)p * m + q] = diff;
        D[(int64_t)q * m + p] = -diff;
      }
    }
    free(buf);
  }
done:
  free(Z);
  free(Hm);
  free(mz);
  free(vz);
  return status;
}

/* Table mode: k_list from the memoised measure matrix.  `want` is ignored
 * (all rows are computed). */
static int lo_step_table(const double* Xc, int64_t n, const int32_t* U, int32_t m,
                         double* k_list) {
  double* D = (double*)malloc(sizeof(double) * (size_t)m * (size_t)m);
  if (!D) return LO_NOMEM;
  const int status = lo_pair_matrix(Xc, n, U, m, D);
  if (!status) {
    for (int32_t p = 0; p < m; ++p) {
      double k = 0.0;
      for (int32_t q = 0; q < m; ++q) {
        if (q == p) continue;
        const double v = D[(int64_t)p * m + q];
        const double neg = v < 0.0 ? v : 0.0;
        k += neg * neg;
      }
      k_list[p] = -k;
    }
  }
  free(D);
  return status;
}

/* R6: x_v <- x_v - (cov(x_v, x_e)/var(x_e)) x_e for v in U, v != e.  Every
 * column is independent of the others, so OpenMP over columns leaves the
 * numbers unchanged. */
static int lo_residualize_cols(double* Xc, int64_t n, const int32_t* U, int32_t m, int32_t e) {
  const double* xe = Xc + (int64_t)e * n;
  const double ve = lo_var(xe, n);
  if (!(ve > 0.0)) return LO_DEGENERATE;
#pragma omp parallel for schedule(static)
  for (int32_t p = 0; p < m; ++p) {
    if (U[p] == e) continue;
    double* xv = Xc + (int64_t)U[p] * n;
    const double b = lo_cov(xv, xe, n) / ve;
    for (int64_t k = 0; k < n; ++k) xv[k] -= b * xe[k];
  }
  return LO_OK;
}

/* Row-major FP32 input (as the GPU receives it) -> FP64 column-major copy. */
static double* lo_load_columns(const float* X, int64_t n, int64_t d, int64_t ldx) {
  double* Xc = (double*)malloc(sizeof(double) * (size_t)n * (size_t)d);
  if (!Xc) return NULL;
  for (int64_t v = 0; v < d; ++v)
    for (int64_t k = 0; k < n; ++k) Xc[v * n + k] = (double)X[k * ldx + v];
  return Xc;
}

/* ------------------------------------------------------------------------ */
/* the full ordering (DirectLiNGAM outer loop, Section 2.2)                  */
/* ------------------------------------------------------------------------ */

/*
 * Steps t0, t0 + 1, ... of the search on a running state, until `nsteps`
 * steps are done or one variable is left:
 *   Xc     FP64 column-major n x d (column v at Xc + v * n): the residual data,
 *          updated in place (R6),
 *   U, m   the active variables (original ids, ascending) and their count,
 *          updated in place; t0 = d - m is the index of the next step.
 * forced  optional (forced_len entries): at step t < forced_len the variable
 *         forced[t] is taken instead of the argmax (teacher forcing); the
 *         measures are still computed and reported.
 * order    out, int32[d]: entry t for every step run; when one variable is
 *          left, entry d - 1 too.
 * measures optional out, double[(d-1) * d]: row t holds k_list of step t by
 *          original column id (NaN for columns already ordered).
 * gaps     optional out, double[d-1]: best minus runner-up of k_list at step t.
 * mode     0 = literal (Algorithm 1 as written), 1 = table (memoised).
 */
static int lo_search_steps(double* Xc, int64_t n, int64_t d, int32_t* U, int32_t* m_io,
                           int32_t nsteps, const int32_t* forced, int32_t forced_len,
                           int32_t mode, int32_t* order, double* measures, double* gaps) {
  double* k_list = (double*)malloc(sizeof(double) * (size_t)d);
  if (!k_list) return LO_NOMEM;
  int32_t m = *m_io;
  int status = LO_OK;
  for (int32_t s = 0; s < nsteps && m > 1; ++s) {
    const int32_t t = (int32_t)d - m;
    status = mode == 1 ? lo_step_table(Xc, n, U, m, k_list)
                       : lo_step_literal(Xc, n, U, m, NULL, k_list);
    if (status) break;
    int32_t best = 0;  /* first maximum (R5) */
    for (int32_t p = 1; p < m; ++p)
      if (k_list[p] > k_list[best]) best = p;
    if (measures) {
      for (int64_t v = 0; v < d; ++v) measures[(int64_t)t * d + v] = NAN;
      for (int32_t p = 0; p < m; ++p) measures[(int64_t)t * d + U[p]] = k_list[p];
    }
    if (gaps) {
      double second = -INFINITY;
      for (int32_t p = 0; p < m; ++p)
        if (p != best && k_list[p] > second) second = k_list[p];
      gaps[t] = k_list[best] - second;
    }
    int32_t chosen = U[best];
    if (t < forced_len) {
      chosen = forced[t];
      int found = 0;
      for (int32_t p = 0; p < m; ++p) found |= (U[p] == chosen);
      if (!found) {
        status = LO_INVALID;
        break;
      }
    }
    order[t] = chosen;
    status = lo_residualize_cols(Xc, n, U, m, chosen);
    if (status) break;
    /* remove `chosen` from U, keeping the ascending order */
    int32_t w = 0;
    for (int32_t p = 0; p < m; ++p)
      if (U[p] != chosen) U[w++] = U[p];
    m = w;
  }
  if (!status && m == 1) order[d - 1] = U[0];
  *m_io = m;
  free(k_list);
  return status;
}

/* The whole ordering (DirectLiNGAM outer loop, Section 2.2) on a column-major
 * FP64 copy that it owns and frees; arguments as for lo_search_steps. */
static int lo_causal_order_cols(double* Xc, int64_t n, int64_t d, const int32_t* forced,
                                int32_t forced_len, int32_t mode, int32_t* order,
                                double* measures, double* gaps) {
  int32_t* U = (int32_t*)malloc(sizeof(int32_t) * (size_t)d);
  if (!Xc || !U) {
    free(Xc);
    free(U);
    return LO_NOMEM;
  }
  for (int32_t v = 0; v < d; ++v) U[v] = v;
  int32_t m = (int32_t)d;
  const int status = lo_search_steps(Xc, n, d, U, &m, (int32_t)d, forced, forced_len, mode,
                                     order, measures, gaps);
  free(Xc);
  free(U);
  return status;
}

/* A search that runs in pieces (long orderings, checkpointed between pieces):
 * the caller owns the state (Xc column-major FP64 n x d, U ascending active
 * ids, *m their count) and calls this with the next `nsteps`; see
 * lo_search_steps.  Free-running (no forcing). */
int lo_causal_order_resume(double* Xc, int64_t n, int64_t d, int32_t* U, int32_t* m,
                           int32_t nsteps, int32_t mode, int32_t* order, double* measures,
                           double* gaps) {
  if (!Xc || !U || !m || !order || n < 2 || d < 1 || *m < 1 || *m > d || nsteps < 0 ||
      (mode != 0 && mode != 1))
    return LO_INVALID;
  for (int32_t p = 0; p < *m; ++p)
    if (U[p] < 0 || U[p] >= d || (p > 0 && U[p] <= U[p - 1])) return LO_INVALID;
  return lo_search_steps(Xc, n, d, U, m, nsteps, NULL, 0, mode, order, measures, gaps);
}

int lo_causal_order(const float* X, int64_t n, int64_t d, int64_t ldx, const int32_t* forced,
                    int32_t forced_len, int32_t mode, int32_t* order, double* measures,
                    double* gaps) {
  if (!X || !order || n < 2 || d < 1 || ldx < d || forced_len < 0 || forced_len > d)
    return LO_INVALID;
  double* Xc = lo_load_columns(X, n, d, ldx);
  if (!Xc) return LO_NOMEM;
  return lo_causal_order_cols(Xc, n, d, forced, forced_len, mode, order, measures, gaps);
}

/* The same on FP64 row-major input (VAR residuals are FP64). */
int lo_causal_order_f64(const double* X, int64_t n, int64_t d, int64_t ldx,
                        const int32_t* forced, int32_t forced_len, int32_t mode, int32_t* order,
                        double* measures, double* gaps) {
  if (!X || !order || n < 2 || d < 1 || ldx < d || forced_len < 0 || forced_len > d)
    return LO_INVALID;
  double* Xc = (double*)malloc(sizeof(double) * (size_t)n * (size_t)d);
  if (!Xc) return LO_NOMEM;
  for (int64_t v = 0; v < d; ++v)
    for (int64_t k = 0; k < n; ++k) Xc[v * n + k] = X[k * ldx + v];
  return lo_causal_order_cols(Xc, n, d, forced, forced_len, mode, order, measures, gaps);
}

/*
 * Measures of selected rows at step t = prefix_len, after regressing out the
 * variables of `prefix` in that order (teacher forcing along a given order).
 * rows / nrows: original column ids whose k_list entry is wanted; each must
 * still be active.  out[r] = k_list entry of rows[r].  Literal mode.
 */
int lo_step_measures_rows(const float* X, int64_t n, int64_t d, int64_t ldx,
                          const int32_t* prefix, int32_t prefix_len, const int32_t* rows,
                          int32_t nrows, double* out) {
  if (!X || !out || n < 2 || d < 2 || ldx < d || prefix_len < 0 || prefix_len > d - 2 ||
      nrows < 0 || (prefix_len > 0 && !prefix) || (nrows > 0 && !rows))
    return LO_INVALID;
  double* Xc = lo_load_columns(X, n, d, ldx);
  int32_t* U = (int32_t*)malloc(sizeof(int32_t) * (size_t)d);
  double* k_list = (double*)malloc(sizeof(double) * (size_t)d);
  unsigned char* want = (unsigned char*)calloc((size_t)d, 1);
  int status = LO_OK;
  if (!Xc || !U || !k_list || !want) {
    status = LO_NOMEM;
    goto done;
  }
  for (int32_t v = 0; v < d; ++v) U[v] = v;
  int32_t m = (int32_t)d;
  for (int32_t t = 0; t < prefix_len; ++t) {
    const int32_t e = prefix[t];
    int found = 0;
    for (int32_t p = 0; p < m; ++p) found |= (U[p] == e);
    if (!found) {
      status = LO_INVALID;
      goto done;
    }
    status = lo_residualize_cols(Xc, n, U, m, e);
    if (status) goto done;
    int32_t w = 0;
    for (int32_t p = 0; p < m; ++p)
      if (U[p] != e) U[w++] = U[p];
    m = w;
  }
  for (int32_t r = 0; r < nrows; ++r) {
    int found = 0;
    for (int32_t p = 0; p < m; ++p)
      if (U[p] == rows[r]) {
        want[p] = 1;
        found = 1;
      }
    if (!found) {
      status = LO_INVALID;
      goto done;
    }
  }
  status = lo_step_literal(Xc, n, U, m, want, k_list);
  if (status) goto done;
  for (int32_t r = 0; r < nrows; ++r)
    for (int32_t p = 0; p < m; ++p)
      if (U[p] == rows[r]) out[r] = k_list[p];
done:
  free(Xc);
  free(U);
  free(k_list);
  free(want);
  return status;
}

/*
 * Every k_list entry of step t = prefix_len in table mode, after regressing
 * out the variables of `prefix` in that order (teacher forcing along a given
 * order): the residualisation of the outer loop (R6) step by step, then one
 * table-mode step (the memoised Algorithm 1) on the active columns.
 *   Xc   FP64 column-major n x d (column v at Xc + v * n), consumed (modified).
 *   out  double[d]: out[v] = k_list entry of v for active v, NaN for the prefix.
 */
static int lo_step_measures_all_cols(double* Xc, int64_t n, int64_t d, const int32_t* prefix,
                                     int32_t prefix_len, double* out) {
  int32_t* U = (int32_t*)malloc(sizeof(int32_t) * (size_t)d);
  double* k_list = (double*)malloc(sizeof(double) * (size_t)d);
  int status = LO_OK;
  if (!U || !k_list) {
    status = LO_NOMEM;
    goto done;
  }
  for (int32_t v = 0; v < d; ++v) U[v] = v;
  int32_t m = (int32_t)d;
  for (int32_t t = 0; t < prefix_len; ++t) {
    const int32_t e = prefix[t];
    int found = 0;
    for (int32_t p = 0; p < m; ++p) found |= (U[p] == e);
    if (!found) {
      status = LO_INVALID;
      goto done;
    }
    status = lo_residualize_cols(Xc, n, U, m, e);
    if (status) goto done;
    int32_t w = 0;
    for (int32_t p = 0; p < m; ++p)
      if (U[p] != e) U[w++] = U[p];
    m = w;
  }
  status = lo_step_table(Xc, n, U, m, k_list);
  if (status) goto done;
  for (int64_t v = 0; v < d; ++v) out[v] = NAN;
  for (int32_t p = 0; p < m; ++p) out[U[p]] = k_list[p];
done:
  free(U);
  free(k_list);
  return status;
}

/* lo_step_measures_all_cols on FP32 row-major input (what the GPU receives). */
int lo_step_measures_all(const float* X, int64_t n, int64_t d, int64_t ldx,
                         const int32_t* prefix, int32_t prefix_len, double* out) {
  if (!X || !out || n < 2 || d < 2 || ldx < d || prefix_len < 0 || prefix_len > d - 2 ||
      (prefix_len > 0 && !prefix))
    return LO_INVALID;
  double* Xc = lo_load_columns(X, n, d, ldx);
  if (!Xc) return LO_NOMEM;
  const int status = lo_step_measures_all_cols(Xc, n, d, prefix, prefix_len, out);
  free(Xc);
  return status;
}

/* The same on FP64 row-major input (VAR residuals are FP64). */
int lo_step_measures_all_f64(const double* X, int64_t n, int64_t d, int64_t ldx,
                             const int32_t* prefix, int32_t prefix_len, double* out) {
  if (!X || !out || n < 2 || d < 2 || ldx < d || prefix_len < 0 || prefix_len > d - 2 ||
      (prefix_len > 0 && !prefix))
    return LO_INVALID;
  double* Xc = (double*)malloc(sizeof(double) * (size_t)n * (size_t)d);
  if (!Xc) return LO_NOMEM;
  for (int64_t v = 0; v < d; ++v)
    for (int64_t k = 0; k < n; ++k) Xc[v * n + k] = X[k * ldx + v];
  const int status = lo_step_measures_all_cols(Xc, n, d, prefix, prefix_len, out);
  free(Xc);
  return status;
}

/* One residualisation on a row-major FP64 matrix (the primitive the library's
 * lingam_residualize entry point implements): for every active column v != exo,
 * x_v <- x_v - (cov(x_v, x_exo)/var(x_exo)) x_exo.  In place. */
int lo_residualize(double* X, int64_t n, int64_t d, int64_t ldx, const int32_t* active,
                   int32_t n_active, int32_t exo) {
  if (!X || !active || n < 2 || d < 1 || ldx < d || n_active < 1 || exo < 0 || exo >= d)
    return LO_INVALID;
  double* xe = (double*)malloc(sizeof(double) * (size_t)n);
  double* xv = (double*)malloc(sizeof(double) * (size_t)n);
  int status = LO_OK;
  if (!xe || !xv) {
    status = LO_NOMEM;
    goto done;
  }
  for (int64_t k = 0; k < n; ++k) xe[k] = X[k * ldx + exo];
  const double ve = lo_var(xe, n);
  if (!(ve > 0.0)) {
    status = LO_DEGENERATE;
    goto done;
  }
  for (int32_t p = 0; p < n_active; ++p) {
    const int32_t v = active[p];
    if (v < 0 || v >= d) {
      status = LO_INVALID;
      goto done;
    }
    if (v == exo) continue;
    for (int64_t k = 0; k < n; ++k) xv[k] = X[k * ldx + v];
    const double b = lo_cov(xv, xe, n) / ve;
    for (int64_t k = 0; k < n; ++k) X[k * ldx + v] = xv[k] - b * xe[k];
  }
done:
  free(xe);
  free(xv);
  return status;
}

/* ------------------------------------------------------------------------ */
/* VarLiNGAM: least-squares VAR(lags) fit with intercept (Section 3.2)       */
/* ------------------------------------------------------------------------ */

/* Cholesky factorisation A = L L^T in place (lower triangle), FP64. */
static int lo_cholesky(double* A, int64_t p) {
  for (int64_t j = 0; j < p; ++j) {
    double s = A[j * p + j];
    for (int64_t k = 0; k < j; ++k) s -= A[j * p + k] * A[j * p + k];
    if (!(s > 0.0)) return LO_DEGENERATE;
    const double l = sqrt(s);
    A[j * p + j] = l;
    for (int64_t i = j + 1; i < p; ++i) {
      double t = A[i * p + j];
      for (int64_t k = 0; k < j; ++k) t -= A[i * p + k] * A[j * p + k];
      A[i * p + j] = t / l;
    }
  }
  return LO_OK;
}

/*
 * X      FP64 row-major T x d series (leading dimension ldx).
 * coef   out, double[(1 + d*lags) * d] row-major: row 0 is the intercept,
 *        row 1 + (tau-1)*d + v is the coefficient of x_v(t - tau).
 * resid  optional out, double[(T - lags) * d] row-major: x(t) - fitted.
 * Solves the normal equations (Z^T Z) A = Z^T Y by Cholesky, Z = [1, x(t-1),
 * ..., x(t-lags)], Y = x(t), t = lags .. T-1.
 */
int lo_var_fit(const double* X, int64_t T, int64_t d, int64_t ldx, int32_t lags, double* coef,
               double* resid) {
  if (!X || !coef || lags < 1 || d < 1 || ldx < d || T <= lags + 1) return LO_INVALID;
  const int64_t N = T - lags, p = 1 + d * lags;
  double* G = (double*)calloc((size_t)(p * p), sizeof(double));
  double* R = (double*)calloc((size_t)(p * d), sizeof(double));
  double* z = (double*)malloc(sizeof(double) * (size_t)p);
  int status = LO_OK;
  if (!G || !R || !z) {
    status = LO_NOMEM;
    goto done;
  }
  for (int64_t t = lags; t < T; ++t) {
    z[0] = 1.0;
    for (int32_t tau = 1; tau <= lags; ++tau)
      for (int64_t v = 0; v < d; ++v) z[1 + (tau - 1) * d + v] = X[(t - tau) * ldx + v];
    for (int64_t a = 0; a < p; ++a) {
      for (int64_t b = 0; b < p; ++b) G[a * p + b] += z[a] * z[b];
      for (int64_t v = 0; v < d; ++v) R[a * d + v] += z[a] * X[t * ldx + v];
    }
  }
  status = lo_cholesky(G, p);
  if (status) goto done;
  for (int64_t v = 0; v < d; ++v) {
    /* forward then backward substitution for column v */
    for (int64_t i = 0; i < p; ++i) {
      double s = R[i * d + v];
      for (int64_t k = 0; k < i; ++k) s -= G[i * p + k] * coef[k * d + v];
      coef[i * d + v] = s / G[i * p + i];
    }
    for (int64_t i = p - 1; i >= 0; --i) {
      double s = coef[i * d + v];
      for (int64_t k = i + 1; k < p; ++k) s -= G[k * p + i] * coef[k * d + v];
      coef[i * d + v] = s / G[i * p + i];
    }
  }
  if (resid) {
    for (int64_t t = lags; t < T; ++t) {
      z[0] = 1.0;
      for (int32_t tau = 1; tau <= lags; ++tau)
        for (int64_t v = 0; v < d; ++v) z[1 + (tau - 1) * d + v] = X[(t - tau) * ldx + v];
      for (int64_t v = 0; v < d; ++v) {
        double f = 0.0;
        for (int64_t a = 0; a < p; ++a) f += z[a] * coef[a * d + v];
        resid[(t - lags) * d + v] = X[t * ldx + v] - f;
      }
    }
  }
  (void)N;
done:
  free(G);
  free(R);
  free(z);
  return status;
}

/* ------------------------------------------------------------------------ */
/* adjacency by least squares on order predecessors                          */
/* ------------------------------------------------------------------------ */

/*
 * E      FP64 row-major n x d (leading dimension lde).
 * order  causal order (original column ids, exogenous first).
 * B      out, double[d * d] row-major: B[c * d + p] is the coefficient of
 *        column p in the least-squares regression (with intercept) of column c
 *        on all columns that precede c in `order`; 0 elsewhere.
 * Each regression solves its own normal equations on centred data by
 * Cholesky (plain, one variable at a time).  This is the instantaneous
 * matrix that VarLiNGAM estimates from the VAR residuals (Section 3.2).
 */
int lo_ols_adjacency(const double* E, int64_t n, int64_t d, int64_t lde, const int32_t* order,
                     double* B) {
  if (!E || !order || !B || n < 2 || d < 1 || lde < d) return LO_INVALID;
  double* mu = (double*)malloc(sizeof(double) * (size_t)d);
  double* C = (double*)malloc(sizeof(double) * (size_t)(d * d));
  int status = LO_OK;
  if (!mu || !C) {
    status = LO_NOMEM;
    goto done;
  }
  for (int64_t v = 0; v < d; ++v) {
    double s = 0.0;
    for (int64_t k = 0; k < n; ++k) s += E[k * lde + v];
    mu[v] = s / (double)n;
  }
  /* covariance matrix (ddof = 0; the scale cancels in the coefficients) */
  for (int64_t a = 0; a < d; ++a)
    for (int64_t b = a; b < d; ++b) {
      double s = 0.0;
      for (int64_t k = 0; k < n; ++k) s += (E[k * lde + a] - mu[a]) * (E[k * lde + b] - mu[b]);
      C[a * d + b] = C[b * d + a] = s / (double)n;
    }
  for (int64_t i = 0; i < d * d; ++i) B[i] = 0.0;
  for (int64_t k = 1; k < d; ++k) {
    const int32_t c = order[k];
    double* G = (double*)malloc(sizeof(double) * (size_t)(k * k));
    double* r = (double*)malloc(sizeof(double) * (size_t)k);
    if (!G || !r) {
      free(G);
      free(r);
      status = LO_NOMEM;
      goto done;
    }
    for (int64_t a = 0; a < k; ++a) {
      for (int64_t b = 0; b < k; ++b) G[a * k + b] = C[(int64_t)order[a] * d + order[b]];
      r[a] = C[(int64_t)order[a] * d + c];
    }
    status = lo_cholesky(G, k);
    if (!status) {
      for (int64_t i = 0; i < k; ++i) {
        double s = r[i];
        for (int64_t q = 0; q < i; ++q) s -= G[i * k + q] * r[q];
        r[i] = s / G[i * k + i];
      }
      for (int64_t i = k - 1; i >= 0; --i) {
        double s = r[i];
        for (int64_t q = i + 1; q < k; ++q) s -= G[q * k + i] * r[q];
        r[i] = s / G[i * k + i];
      }
      for (int64_t a = 0; a < k; ++a) B[(int64_t)c * d + order[a]] = r[a];
    }
    free(G);
    free(r);
    if (status) goto done;
  }
done:
  free(mu);
  free(C);
  return status;
}

/* number of OpenMP threads the oracle will use */
int lo_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/*
 * FP64 CPU oracle for the averaged randomized sparse Kaczmarz method (RSKA).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test-suite, the smoke entry and the CPU
 * baseline leg of the benchmark may load this library. It shares no code,
 * header, table or helper with the HIP implementation.
 *
 * Everything is plain double-precision loops in the order the paper states:
 *   - the RSKA iteration, eq. (rska) in Sec. 1.1 and Algorithm 1 (RSKA):
 *       x*_{k+1} = x*_k - (1/eta) sum_{i in tau_k} w_i (<a_i,x_k> - b_i)/||a_i||^2 a_i
 *       x_{k+1}  = S_lambda(x*_{k+1}),  x_0 = x*_0 = 0
 *     with uniform weights w_i = alpha (variant v2 of Sec. 5), or a per-step
 *     alpha_k when one is given;
 *   - the soft shrinkage S_lambda(x) = max(|x|-lambda, 0) sign(x) (Sec. 1.1);
 *   - the dual variable y with x* = A^T y, which the update keeps by
 *     construction (the sketch-and-project form, eq. (rska1), and the start of
 *     Sec. 4): y_i -= c_t for every sampled row i = tau_k[t].
 * The index multiset tau_k is an input (eta indices per step, drawn with
 * replacement; duplicates are counted each time), so the oracle contains no
 * random number generator.
 *
 * Readings of points the paper leaves open (all residuals of one step use the
 * same x_k; delta is formed before it is subtracted; j ascending in dots and t
 * ascending in the column sums) are listed with the design notes.
 *
 * Return codes: 0 ok, 1 invalid argument, 5 zero-norm row referenced,
 * 6 index out of range, 7 non-finite iterate.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_INVALID 1
#define OR_ZERO_ROW 5
#define OR_INDEX 6
#define OR_NONFINITE 7

/* Soft shrinkage, Sec. 1.1. |v| == lambda gives 0. */
static double shrink(double v, double lambda) {
  double a = fabs(v) - lambda;
  if (a <= 0.0) return 0.0;
  return v > 0.0 ? a : -a;
}

/* ||a_i||^2 for every row of a dense row-major matrix (Def. 1, the matrix D). */
int oracle_rownorm2_dense(int64_t m, int64_t n, int64_t ld, const double *A, double *r2) {
  if (m < 0 || n < 0 || ld < n || (m > 0 && (!A || !r2))) return OR_INVALID;
  for (int64_t i = 0; i < m; ++i) {
    double s = 0.0;
    for (int64_t j = 0; j < n; ++j) s += A[i * ld + j] * A[i * ld + j];
    r2[i] = s;
  }
  return OR_OK;
}

int oracle_rownorm2_csr(int64_t m, const int64_t *row_ptr, const double *val, double *r2) {
  if (m < 0 || (m > 0 && (!row_ptr || !r2))) return OR_INVALID;
  for (int64_t i = 0; i < m; ++i) {
    double s = 0.0;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) s += val[p] * val[p];
    r2[i] = s;
  }
  return OR_OK;
}

/* Shared argument checks of the two solvers. */
static int check_common(int64_t m, int64_t n, double lambda, int32_t eta, double alpha,
                        const double *alpha_k, int64_t K, const int32_t *idx, const double *b,
                        double *z, double *x) {
  if (m <= 0 || n <= 0 || eta < 1 || K < 0) return OR_INVALID;
  if (!(lambda >= 0.0) || !isfinite(lambda)) return OR_INVALID;
  if (!alpha_k && (!(alpha > 0.0) || !isfinite(alpha))) return OR_INVALID;
  if (!b || !z || !x || (K > 0 && !idx)) return OR_INVALID;
  return OR_OK;
}

/* Relative error ||x - xref|| / ||xref|| (the error measure of Sec. 5). */
static double rel_err(int64_t n, const double *x, const double *xref) {
  double num = 0.0, den = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    double d = x[j] - xref[j];
    num += d * d;
    den += xref[j] * xref[j];
  }
  return den > 0.0 ? sqrt(num / den) : sqrt(num);
}

/*
 * Dense RSKA. A is m x n row-major with leading dimension ld.
 * z (= x*) is in/out: the run starts from the given z (pass zeros for the
 * paper's x*_0 = 0) and x_0 = S_lambda(z). x receives S_lambda(z_K).
 * y (nullable, length m) is in/out: y[i_t] -= c_t each step.
 * Step k uses indices idx[off + k*eta + t], t = 0..eta-1, and the relaxation
 * alpha_k[k] if alpha_k is given, else alpha, times row_w[i] for row i when
 * row_w (length m) is given: the diagonal weight matrix W of Definition 1
 * (variants v3/v4 of Sec. 5), c_t = (w_i / eta) (<a_i, x> - b_i) / ||a_i||^2.
 * If check_every > 0 and xref/err_hist are given, err_hist[q] receives the
 * relative error after step (q+1)*check_every.
 * *k_done receives the number of completed steps (nullable).
 *
 * nthreads > 1 spreads the eta residuals of a step (independent of each
 * other: Algorithm 1 computes them "in parallel" at the same x_k) and the
 * columns of delta_k over threads. No sum changes its order: every dot runs j
 * ascending inside one thread, and every delta_j runs t ascending inside the
 * thread that owns column j. The result is the same bits for any nthreads.
 */
int oracle_rska_dense_threads(int64_t m, int64_t n, int64_t ld, const double *A, const double *b,
                              double lambda, int32_t eta, double alpha, const double *alpha_k,
                              const double *row_w, int64_t K, const int32_t *idx, int64_t off,
                              double *z, double *x, double *y,
                              int64_t check_every, const double *xref, double *err_hist,
                              int64_t *k_done, int32_t nthreads) {
  int st = check_common(m, n, lambda, eta, alpha, alpha_k, K, idx, b, z, x);
  if (st) return st;
  if (!A || ld < n) return OR_INVALID;
  if (nthreads < 1) nthreads = 1;
  if (k_done) *k_done = 0;
  double *c = (double *)malloc(sizeof(double) * (size_t)eta);
  double *rn = (double *)malloc(sizeof(double) * (size_t)eta);
  double *delta = (double *)malloc(sizeof(double) * (size_t)n);
  if (!c || !rn || !delta) { free(c); free(rn); free(delta); return OR_INVALID; }

  for (int64_t j = 0; j < n; ++j) x[j] = shrink(z[j], lambda);
  for (int64_t k = 0; k < K; ++k) {
    const int32_t *tau = idx + off + k * (int64_t)eta;
    double ak = alpha_k ? alpha_k[k] : alpha;
    /* residuals of all eta rows at the same x_k, then the coefficients */
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 4) if (nthreads > 1)
    for (int32_t t = 0; t < eta; ++t) {
      int64_t i = tau[t];
      rn[t] = -1.0;
      if (i < 0 || i >= m) continue;
      const double *ai = A + i * ld;
      double r2 = 0.0, dot = 0.0;
      for (int64_t j = 0; j < n; ++j) r2 += ai[j] * ai[j];
      for (int64_t j = 0; j < n; ++j) dot += ai[j] * x[j];
      rn[t] = r2;
      if (r2 != 0.0) c[t] = ((row_w ? ak * row_w[i] : ak) / (double)eta) * (dot - b[i]) / r2;
    }
    /* the first bad row in t order decides the error */
    for (int32_t t = 0; t < eta; ++t) {
      if (tau[t] < 0 || tau[t] >= m) { st = OR_INDEX; goto done; }
      if (rn[t] == 0.0) { st = OR_ZERO_ROW; goto done; }
    }
    /* delta_k = sum_t c_t a_{tau_t}, formed first, then subtracted */
#pragma omp parallel num_threads(nthreads) if (nthreads > 1)
    {
#ifdef _OPENMP
      const int nth = omp_get_num_threads(), me = omp_get_thread_num();
#else
      const int nth = 1, me = 0;
#endif
      const int64_t per = ((n + nth - 1) / nth + 7) / 8 * 8;
      const int64_t j0 = per * me < n ? per * me : n, j1 = j0 + per < n ? j0 + per : n;
      for (int64_t j = j0; j < j1; ++j) delta[j] = 0.0;
      for (int32_t t = 0; t < eta; ++t) {
        const double *ai = A + (int64_t)tau[t] * ld;
        for (int64_t j = j0; j < j1; ++j) delta[j] += c[t] * ai[j];
      }
    }
    int finite = 1;
    for (int64_t j = 0; j < n; ++j) {
      z[j] -= delta[j];
      x[j] = shrink(z[j], lambda);
      if (!isfinite(z[j])) finite = 0;
    }
    if (y)
      for (int32_t t = 0; t < eta; ++t) y[tau[t]] -= c[t];
    if (k_done) *k_done = k + 1;
    if (!finite) { st = OR_NONFINITE; goto done; }
    if (check_every > 0 && xref && err_hist && (k + 1) % check_every == 0)
      err_hist[(k + 1) / check_every - 1] = rel_err(n, x, xref);
  }
done:
  free(c);
  free(rn);
  free(delta);
  return st;
}

int oracle_rska_dense(int64_t m, int64_t n, int64_t ld, const double *A, const double *b,
                      double lambda, int32_t eta, double alpha, const double *alpha_k,
                      const double *row_w, int64_t K, const int32_t *idx, int64_t off,
                      double *z, double *x, double *y,
                      int64_t check_every, const double *xref, double *err_hist,
                      int64_t *k_done) {
  return oracle_rska_dense_threads(m, n, ld, A, b, lambda, eta, alpha, alpha_k, row_w, K, idx, off, z, x, y,
                                   check_every, xref, err_hist, k_done, 1);
}

/*
 * CSR RSKA: the same iteration with the rows stored as (row_ptr, col, val).
 * Column indices of a row need not be sorted; repeated columns add up.
 */
int oracle_rska_csr(int64_t m, int64_t n, const int64_t *row_ptr, const int32_t *col,
                    const double *val, const double *b,
                    double lambda, int32_t eta, double alpha, const double *alpha_k,
                    const double *row_w, int64_t K, const int32_t *idx, int64_t off,
                    double *z, double *x, double *y,
                    int64_t check_every, const double *xref, double *err_hist,
                    int64_t *k_done) {
  int st = check_common(m, n, lambda, eta, alpha, alpha_k, K, idx, b, z, x);
  if (st) return st;
  if (!row_ptr || !col || !val) return OR_INVALID;
  if (k_done) *k_done = 0;
  double *c = (double *)malloc(sizeof(double) * (size_t)eta);
  double *delta = (double *)malloc(sizeof(double) * (size_t)n);
  if (!c || !delta) { free(c); free(delta); return OR_INVALID; }

  for (int64_t j = 0; j < n; ++j) x[j] = shrink(z[j], lambda);
  for (int64_t k = 0; k < K; ++k) {
    const int32_t *tau = idx + off + k * (int64_t)eta;
    double ak = alpha_k ? alpha_k[k] : alpha;
    for (int32_t t = 0; t < eta; ++t) {
      int64_t i = tau[t];
      if (i < 0 || i >= m) { st = OR_INDEX; goto done; }
      double r2 = 0.0, dot = 0.0;
      for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        if (col[p] < 0 || col[p] >= n) { st = OR_INDEX; goto done; }
        r2 += val[p] * val[p];
        dot += val[p] * x[col[p]];
      }
      if (r2 == 0.0) { st = OR_ZERO_ROW; goto done; }
      c[t] = ((row_w ? ak * row_w[i] : ak) / (double)eta) * (dot - b[i]) / r2;
    }
    for (int64_t j = 0; j < n; ++j) delta[j] = 0.0;
    for (int32_t t = 0; t < eta; ++t) {
      int64_t i = tau[t];
      for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) delta[col[p]] += c[t] * val[p];
    }
    int finite = 1;
    for (int64_t j = 0; j < n; ++j) {
      z[j] -= delta[j];
      x[j] = shrink(z[j], lambda);
      if (!isfinite(z[j])) finite = 0;
    }
    if (y)
      for (int32_t t = 0; t < eta; ++t) y[tau[t]] -= c[t];
    if (k_done) *k_done = k + 1;
    if (!finite) { st = OR_NONFINITE; goto done; }
    if (check_every > 0 && xref && err_hist && (k + 1) % check_every == 0)
      err_hist[(k + 1) / check_every - 1] = rel_err(n, x, xref);
  }
done:
  free(c);
  free(delta);
  return st;
}

/*
 * Reverse mode of K unrolled dense RSKA steps from z_0 = 0, for one right-hand
 * side. The forward map is the iteration above with per-step relaxations
 * alpha_k[k]; the loss gradient with respect to x_K is given (xbar_K).
 * All K+1 iterates z_k are stored (no checkpointing: this is the plain
 * definition of the chain rule, taken step by step backwards):
 *   z_{k+1} = z_k - A_k^T c_k,   c_{k,t} = (alpha_k/eta) (a_t.x_k - b_t)/r2_t,
 *   x_k = S_lambda(z_k),  dS/dz = 1[|z| > lambda],  dS/dlambda = -sign(z) 1[|z| > lambda].
 * Outputs: bbar (m, accumulated: +=), *lambda_bar (+=), alpha_bar (K, +=).
 */
int oracle_rska_dense_adjoint(int64_t m, int64_t n, int64_t ld, const double *A, const double *b,
                              double lambda, int32_t eta, const double *alpha_k,
                              int64_t K, const int32_t *idx, int64_t off,
                              const double *xbar_K,
                              double *bbar, double *lambda_bar, double *alpha_bar) {
  if (m <= 0 || n <= 0 || eta < 1 || K < 0 || !A || ld < n || !b || !alpha_k || !xbar_K ||
      !bbar || !lambda_bar || !alpha_bar || (K > 0 && !idx) || !(lambda >= 0.0))
    return OR_INVALID;
  int st = OR_OK;
  double *Z = (double *)calloc((size_t)(K + 1) * (size_t)n, sizeof(double));
  double *xk = (double *)malloc(sizeof(double) * (size_t)n);
  double *zbar = (double *)malloc(sizeof(double) * (size_t)n);
  double *xbar = (double *)malloc(sizeof(double) * (size_t)n);
  double *r = (double *)malloc(sizeof(double) * (size_t)eta);
  double *r2 = (double *)malloc(sizeof(double) * (size_t)eta);
  double *cbar = (double *)malloc(sizeof(double) * (size_t)eta);
  if (!Z || !xk || !zbar || !xbar || !r || !r2 || !cbar) { st = OR_INVALID; goto done; }

  /* forward, storing every z_k */
  for (int64_t k = 0; k < K; ++k) {
    const int32_t *tau = idx + off + k * (int64_t)eta;
    double *zk = Z + k * n, *zn = Z + (k + 1) * n;
    for (int64_t j = 0; j < n; ++j) { xk[j] = shrink(zk[j], lambda); zn[j] = zk[j]; }
    for (int32_t t = 0; t < eta; ++t) {
      int64_t i = tau[t];
      if (i < 0 || i >= m) { st = OR_INDEX; goto done; }
      const double *ai = A + i * ld;
      double s2 = 0.0, dot = 0.0;
      for (int64_t j = 0; j < n; ++j) { s2 += ai[j] * ai[j]; dot += ai[j] * xk[j]; }
      if (s2 == 0.0) { st = OR_ZERO_ROW; goto done; }
      double ct = (alpha_k[k] / (double)eta) * (dot - b[i]) / s2;
      for (int64_t j = 0; j < n; ++j) zn[j] -= ct * ai[j];
    }
  }
  /* seed: x_K = S(z_K) */
  {
    const double *zK = Z + K * n;
    for (int64_t j = 0; j < n; ++j) {
      int on = fabs(zK[j]) > lambda;
      zbar[j] = on ? xbar_K[j] : 0.0;
      if (on) *lambda_bar -= (zK[j] > 0.0 ? 1.0 : -1.0) * xbar_K[j];
    }
  }
  /* backwards through the steps */
  for (int64_t k = K - 1; k >= 0; --k) {
    const int32_t *tau = idx + off + k * (int64_t)eta;
    const double *zk = Z + k * n;
    for (int64_t j = 0; j < n; ++j) xk[j] = shrink(zk[j], lambda);
    double abar = 0.0;
    for (int32_t t = 0; t < eta; ++t) {
      const double *ai = A + (int64_t)tau[t] * ld;
      double s2 = 0.0, dot = 0.0, g = 0.0;
      for (int64_t j = 0; j < n; ++j) { s2 += ai[j] * ai[j]; dot += ai[j] * xk[j]; g += ai[j] * zbar[j]; }
      r[t] = dot - b[tau[t]];
      r2[t] = s2;
      cbar[t] = -g;                                   /* dL/dc_t = -<a_t, zbar_{k+1}> */
      abar += cbar[t] * r[t] / ((double)eta * s2);    /* dc_t/dalpha_k */
    }
    alpha_bar[k] += abar;
    for (int64_t j = 0; j < n; ++j) xbar[j] = 0.0;
    for (int32_t t = 0; t < eta; ++t) {
      double rbar = cbar[t] * alpha_k[k] / ((double)eta * r2[t]);
      bbar[tau[t]] -= rbar;                           /* r_t = a_t.x_k - b_t */
      const double *ai = A + (int64_t)tau[t] * ld;
      for (int64_t j = 0; j < n; ++j) xbar[j] += rbar * ai[j];
    }
    for (int64_t j = 0; j < n; ++j) {
      if (fabs(zk[j]) > lambda) {
        zbar[j] += xbar[j];
        *lambda_bar -= (zk[j] > 0.0 ? 1.0 : -1.0) * xbar[j];
      }
    }
  }
done:
  free(Z); free(xk); free(zbar); free(xbar); free(r); free(r2); free(cbar);
  return st;
}

/*
 * Row sampler (the index stream of Sec. 1.1 drawn from a counter-based
 * generator instead of being handed in).
 *
 * Philox4x32-10 as defined by Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3" (SC'11): the 128-bit counter passes through ten
 * rounds; a round multiplies words 0 and 2 by M0 = 0xD2511F53 and
 * M1 = 0xCD9E8D57 into 64-bit products and outputs
 *   (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0));
 * between rounds the key is advanced by the Weyl constants W0 = 0x9E3779B9,
 * W1 = 0xBB67AE85 (the first round uses the key as given).
 */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* cdf_i = w_0 + ... + w_i, i ascending (sampling weights w_i = ||a_i||^2). */
int oracle_sampling_cdf(int64_t m, const double *w, double *cdf) {
  if (m <= 0 || !w || !cdf) return 1;
  double s = 0.0;
  for (int64_t i = 0; i < m; ++i) {
    if (!(w[i] >= 0.0)) return 1;
    s += w[i];
    cdf[i] = s;
  }
  return 0;
}

/*
 * Index t of step k (k0 <= k < k0 + K, 0 <= t < eta): Philox4x32-10 of the
 * counter (t, k mod 2^32, k div 2^32, 0) under the key (seed mod 2^32,
 * seed div 2^32) gives words w0, w1; u = ((w0 >> 5) 2^26 + (w1 >> 6)) / 2^53
 * in [0, 1); the row is the first i with cdf_i > u cdf_{m-1} (at most m-1),
 * so P(i) = w_i / sum_j w_j (sampling with replacement, p_i proportional to
 * ||a_i||^2). out[(k - k0) eta + t], step-major.
 */
int oracle_sample_stream(int64_t m, const double *cdf, uint64_t seed, int64_t k0, int64_t K, int32_t eta,
                         int32_t *out) {
  if (m <= 0 || !cdf || K < 0 || k0 < 0 || eta < 1 || (K > 0 && !out)) return 1;
  const double total = cdf[m - 1];
  if (!(total > 0.0) || !isfinite(total)) return 1;
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int64_t k = k0; k < k0 + K; ++k) {
    for (int32_t t = 0; t < eta; ++t) {
      const uint32_t ctr[4] = {(uint32_t)t, (uint32_t)k, (uint32_t)((uint64_t)k >> 32), 0u};
      uint32_t w[4];
      oracle_philox4x32_10(ctr, key, w);
      const uint64_t bits = ((uint64_t)(w[0] >> 5) << 26) | (uint64_t)(w[1] >> 6);
      const double u = (double)bits * (1.0 / 9007199254740992.0);
      const double target = u * total;
      /* first i with cdf[i] > target */
      int64_t lo = 0, hi = m;
      while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (cdf[mid] > target) hi = mid;
        else lo = mid + 1;
      }
      out[(k - k0) * eta + t] = (int32_t)(lo < m ? lo : m - 1);
    }
  }
  return 0;
}

/*
 * Linearized Bregman method (full-batch comparator; the remark on its
 * convergence rate in Sec. 4, and eq. (bsk) with tau_k = all rows):
 *   x*_{k+1} = x*_k - s A^T (A x_k - b),  x_{k+1} = S_lambda(x*_{k+1}),
 * with step s (1/||A||_2^2 in the paper). r = A x - b is formed first, then
 * A^T r (j ascending, i ascending). Optional monitor as in oracle_rska_dense,
 * and the residual norm ||A x_k - b|| of every step in res_hist (nullable).
 */
int oracle_lb_dense(int64_t m, int64_t n, int64_t ld, const double *A, const double *b, double lambda, double step,
                    int64_t K, double *z, double *x, int64_t check_every, const double *xref, double *err_hist,
                    double *res_hist) {
  if (m <= 0 || n <= 0 || ld < n || !A || !b || !z || !x || K < 0 || !(lambda >= 0.0) || !(step > 0.0)) return 1;
  double *r = (double *)malloc(sizeof(double) * (size_t)m);
  double *g = (double *)malloc(sizeof(double) * (size_t)n);
  if (!r || !g) { free(r); free(g); return 1; }
  for (int64_t j = 0; j < n; ++j) { z[j] = 0.0; x[j] = 0.0; }
  int code = 0;
  for (int64_t k = 0; k < K; ++k) {
    double rr = 0.0;
    for (int64_t i = 0; i < m; ++i) {
      double s = 0.0;
      for (int64_t j = 0; j < n; ++j) s += A[i * ld + j] * x[j];
      r[i] = s - b[i];
      rr += r[i] * r[i];
    }
    if (res_hist) res_hist[k] = sqrt(rr);
    for (int64_t j = 0; j < n; ++j) g[j] = 0.0;
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < n; ++j) g[j] += A[i * ld + j] * r[i];
    for (int64_t j = 0; j < n; ++j) {
      z[j] -= step * g[j];
      x[j] = shrink(z[j], lambda);
      if (!isfinite(z[j])) code = 7;
    }
    if (code) break;
    if (xref && check_every > 0 && (k + 1) % check_every == 0 && err_hist)
      err_hist[(k + 1) / check_every - 1] = rel_err(n, x, xref);
  }
  free(r);
  free(g);
  return code;
}

/* sigma_max(A)^2 by `iters` steps of power iteration on A^T A from v0 (n):
   w = A^T (A v), estimate = <v, w> with ||v|| = 1, then v = w / ||w||. */
int oracle_power_ata(int64_t m, int64_t n, int64_t ld, const double *A, int64_t iters, const double *v0,
                     double *est) {
  if (m <= 0 || n <= 0 || ld < n || !A || !v0 || !est || iters < 1) return 1;
  double *v = (double *)malloc(sizeof(double) * (size_t)n);
  double *w = (double *)malloc(sizeof(double) * (size_t)n);
  double *u = (double *)malloc(sizeof(double) * (size_t)m);
  if (!v || !w || !u) { free(v); free(w); free(u); return 1; }
  double nv = 0.0;
  for (int64_t j = 0; j < n; ++j) nv += v0[j] * v0[j];
  nv = sqrt(nv);
  for (int64_t j = 0; j < n; ++j) v[j] = v0[j] / nv;
  double lam = 0.0;
  for (int64_t it = 0; it < iters; ++it) {
    for (int64_t i = 0; i < m; ++i) {
      double s = 0.0;
      for (int64_t j = 0; j < n; ++j) s += A[i * ld + j] * v[j];
      u[i] = s;
    }
    for (int64_t j = 0; j < n; ++j) w[j] = 0.0;
    for (int64_t i = 0; i < m; ++i)
      for (int64_t j = 0; j < n; ++j) w[j] += A[i * ld + j] * u[i];
    double vw = 0.0, ww = 0.0;
    for (int64_t j = 0; j < n; ++j) { vw += v[j] * w[j]; ww += w[j] * w[j]; }
    lam = vw;
    ww = sqrt(ww);
    if (!(ww > 0.0)) break;
    for (int64_t j = 0; j < n; ++j) v[j] = w[j] / ww;
  }
  *est = lam;
  free(v); free(w); free(u);
  return 0;
}

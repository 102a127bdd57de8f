/*
 * spectral_big.c -- equal-size MLE loss of the multitask GP on digital nets,
 * and the dense posterior-mean sum, in plain C (float64, OpenMP threads) for
 * sizes where the numpy spectral oracle would need minutes and tens of GB.
 *
 * TEST INFRASTRUCTURE ONLY: called from the tests and nowhere else.  It
 * shares no code with the HIP library.  Every step is the plain definition:
 *
 *  - points (Def. "Base-2 digitally-shifted digital sequences"): z_i is the
 *    XOR of the generating columns g_p over the set bits p of i, taken bit by
 *    bit; task t's point i is z_i XOR Delta_t;
 *  - DSI kernels (Eq. DSI_kernel_1d_ex) with beta(x) = -floor(log2 x),
 *    t_nu(x) = 2^(-nu beta(x)) and beta(0) = t_nu(0) = 0; order 1 read as
 *    1 - 3 t_1 (the zero-mean order-one Walsh kernel); the order-4 digit
 *    series over the 32 given digits plus the tail of the zero digits;
 *    the product kernel (Eq. prod_kernel) gamma prod_j (1 + eta_j K(u_j));
 *  - Theorem "Fast MTGP computations" at equal sizes: block (t, u) of the
 *    Gram matrix is the dyadic convolution with c_tu[i] = Q(z_i XOR Delta_t
 *    XOR Delta_u), its eigenvalues are the unnormalised Walsh-Hadamard
 *    transform lambda_tu = H c_tu, and with yhat_t = H y_t / sqrt(n)
 *      Lambda(f)_tu = R_tu lambda_tu(f) + delta_tu xi_t,
 *      L = sum_f rhat(f)^T Lambda(f)^-1 rhat(f) + log det Lambda(f),
 *      rhat_t(f) = yhat_t(f) - [f = 0] sqrt(n) tau_t
 *    (Eq. MTGP_MLE_GCV_loss); profiled means solve the normal equations of
 *    Eq. MTGP_optimal_tau, which involve frequency 0 only:
 *      n Lambda(0)^-1 tau = sqrt(n) Lambda(0)^-1 yhat(0);
 *  - alpha = Ktilde^-1 r per task: alpha_t = H ahat_t / sqrt(n) with
 *    ahat(f) = Lambda(f)^-1 rhat(f);
 *  - the posterior mean (Eq. MTGP_post_mean_cov) as the plain sum
 *      mu(t, x) = tau_t + sum_u R_tu sum_k Q(x XOR x_uk) alpha_uk.
 *
 * Lambda(f) is factored by a textbook Cholesky decomposition; sums over
 * frequencies and over training points accumulate in long double.
 *
 * Pinned (tests/test_oracle_spectral_big.py) against oracle.dense on small
 * designs: every DSI order, fixed and profiled means, T = 1..5, and the
 * posterior mean against oracle.dense.posterior_mean; the points against
 * oracle.points; the target sums against workloads.target_values.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SB_MAXT 16

/* beta(u 2^-32) = -floor(log2(u 2^-32)) for u > 0: the position (1-based,
 * from the most significant) of the leading 1 digit; beta(0) = 0. */
static int sb_beta(uint32_t u) {
  if (u == 0) return 0;
  int b = 1;
  while (!(u & 0x80000000u)) {
    u <<= 1;
    b++;
  }
  return b;
}

/* sum_{a>=1} (1 - 2 x_a) 8^-(a-1) over the binary digits x_a of u 2^-32 */
static double sb_digit_series(uint32_t u) {
  double s = 0.0, w = 1.0;
  for (int a = 1; a <= 32; a++) {
    const int xa = (u >> (32 - a)) & 1u;
    s += (1.0 - 2.0 * xa) * w;
    w /= 8.0;
  }
  return s + (8.0 / 7.0) * w; /* digits beyond the 32nd are zero */
}

static double sb_khat(int order, uint32_t u) {
  const double x = (double)u * 0x1p-32;
  const int bi = sb_beta(u);
  const double b = (double)bi;
  const double t1 = bi ? ldexp(1.0, -bi) : 0.0;
  const double t2 = bi ? ldexp(1.0, -2 * bi) : 0.0;
  const double t3 = bi ? ldexp(1.0, -3 * bi) : 0.0;
  switch (order) {
    case 1: return 6.0 * (1.0 / 6.0 - 0.5 * t1);
    case 2: return -1.0 - b * x + 2.5 * (1.0 - t1);
    case 3: return -1.0 + b * x * x - 5.0 * (1.0 - t1) * x + (43.0 / 18.0) * (1.0 - t2);
    default:
      return -1.0 - (2.0 / 3.0) * b * x * x * x + 5.0 * (1.0 - t1) * x * x -
             (43.0 / 9.0) * (1.0 - t2) * x + (701.0 / 294.0) * (1.0 - t3) +
             b * (sb_digit_series(u) / 48.0 - 1.0 / 42.0);
  }
}

static double sb_q(int d, int order, double gamma, const double* eta, const uint32_t* u) {
  double q = gamma;
  for (int j = 0; j < d; j++) q *= 1.0 + eta[j] * sb_khat(order, u[j]);
  return q;
}

/* z_i (unshifted) for i < n, [n][d]; gen is [d][32] */
int sb_points(const uint32_t* gen, int d, int64_t n, uint32_t* z) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; i++)
    for (int j = 0; j < d; j++) {
      uint32_t v = 0;
      for (int p = 0; p < 32; p++)
        if ((i >> p) & 1) v ^= gen[32 * j + p];
      z[i * d + j] = v;
    }
  return 0;
}

/* unnormalised Walsh-Hadamard transform in place (natural Sylvester order) */
static void sb_walsh(double* x, int64_t n) {
  for (int64_t h = 1; h < n; h *= 2)
    for (int64_t i = 0; i < n; i += 2 * h)
      for (int64_t k = i; k < i + h; k++) {
        const double a = x[k], b = x[k + h];
        x[k] = a + b;
        x[k + h] = a - b;
      }
}

/* Cholesky A = L L^T of a T x T symmetric matrix (lower triangle, row-major,
 * in place); returns 0, or 1 if a pivot is not positive */
static int sb_chol(double* A, int T) {
  for (int j = 0; j < T; j++) {
    double s = A[j * T + j];
    for (int k = 0; k < j; k++) s -= A[j * T + k] * A[j * T + k];
    if (!(s > 0.0)) return 1;
    const double l = sqrt(s);
    A[j * T + j] = l;
    for (int i = j + 1; i < T; i++) {
      double v = A[i * T + j];
      for (int k = 0; k < j; k++) v -= A[i * T + k] * A[j * T + k];
      A[i * T + j] = v / l;
    }
  }
  return 0;
}

/* solves L L^T x = b in place */
static void sb_chol_solve(const double* L, int T, double* b) {
  for (int i = 0; i < T; i++) {
    double v = b[i];
    for (int k = 0; k < i; k++) v -= L[i * T + k] * b[k];
    b[i] = v / L[i * T + i];
  }
  for (int i = T - 1; i >= 0; i--) {
    double v = b[i];
    for (int k = i + 1; k < T; k++) v -= L[k * T + i] * b[k];
    b[i] = v / L[i * T + i];
  }
}

/* Equal-size MLE pieces on a digital net: T tasks of n = 2^m points, data y
 * [T][n] in radical-inverse order.  R is the T x T task covariance
 * (row-major).  out3 = (quad, logdet, L); tau_hat[T] receives the means used
 * (profiled, or tau_in); alpha (may be NULL) receives Ktilde^-1 r as [T][n].
 * Returns 0, 1 (a pivot not positive), 2 (bad arguments), 3 (no memory). */
int sb_mle_equal(int T, int d, int m, const uint32_t* gen, const uint32_t* shift, int order,
                 double gamma, const double* eta, const double* xi, const double* R,
                 int profile, const double* tau_in, const double* y, double* out3,
                 double* tau_hat, double* alpha) {
  if (T < 1 || T > SB_MAXT || d < 1 || m < 0 || m > 30 || order < 1 || order > 4) return 2;
  const int64_t n = (int64_t)1 << m;
  const int npair = T * (T + 1) / 2;
  uint32_t* z = (uint32_t*)malloc((size_t)n * d * sizeof(uint32_t));
  /* one spectrum per distinct column: index 0 the shared diagonal column
   * (pair shift 0), then the pairs t < u */
  const int ncol = 1 + T * (T - 1) / 2;
  double* lam = (double*)malloc((size_t)ncol * n * sizeof(double));
  double* yh = (double*)malloc((size_t)T * n * sizeof(double));
  if (!z || !lam || !yh) {
    free(z);
    free(lam);
    free(yh);
    return 3;
  }
  int colof[SB_MAXT][SB_MAXT];
  uint32_t cshift[1 + SB_MAXT * (SB_MAXT - 1) / 2][64];
  if (d > 64) {
    free(z);
    free(lam);
    free(yh);
    return 2;
  }
  int c = 1;
  for (int j = 0; j < d; j++) cshift[0][j] = 0u;
  for (int t = 0; t < T; t++) {
    colof[t][t] = 0;
    for (int u = t + 1; u < T; u++) {
      colof[t][u] = colof[u][t] = c;
      for (int j = 0; j < d; j++) cshift[c][j] = shift[t * d + j] ^ shift[u * d + j];
      c++;
    }
  }
  (void)npair;
  sb_points(gen, d, n, z);
  /* kernel columns c[i] = Q(z_i XOR s) and their Walsh transforms */
#pragma omp parallel for schedule(dynamic, 1)
  for (int cc = 0; cc < ncol; cc++) {
    double* col = lam + (size_t)cc * n;
    uint32_t u[64];
    for (int64_t i = 0; i < n; i++) {
      for (int j = 0; j < d; j++) u[j] = z[i * d + j] ^ cshift[cc][j];
      col[i] = sb_q(d, order, gamma, eta, u);
    }
    sb_walsh(col, n);
  }
  free(z);
  const double sn = sqrt((double)n);
#pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < T; t++) {
    double* v = yh + (size_t)t * n;
    memcpy(v, y + (size_t)t * n, (size_t)n * sizeof(double));
    sb_walsh(v, n);
    for (int64_t f = 0; f < n; f++) v[f] /= sn;
  }
  /* means: frequency 0 only */
  {
    double A[SB_MAXT * SB_MAXT], b[SB_MAXT];
    for (int t = 0; t < T; t++)
      for (int u = 0; u < T; u++)
        A[t * T + u] = R[t * T + u] * lam[(size_t)colof[t][u] * n] + (t == u ? xi[t] : 0.0);
    if (profile) {
      /* n Lambda(0)^-1 tau = sqrt(n) Lambda(0)^-1 yhat(0): with
       * M = Lambda(0)^-1, tau = (n M)^-1 sqrt(n) M yhat(0) */
      double L0[SB_MAXT * SB_MAXT], Minv[SB_MAXT * SB_MAXT];
      memcpy(L0, A, sizeof(double) * T * T);
      if (sb_chol(L0, T)) {
        free(lam);
        free(yh);
        return 1;
      }
      for (int k = 0; k < T; k++) {
        double e[SB_MAXT] = {0};
        e[k] = 1.0;
        sb_chol_solve(L0, T, e);
        for (int i = 0; i < T; i++) Minv[i * T + k] = e[i];
      }
      double rhs[SB_MAXT], N0[SB_MAXT * SB_MAXT];
      for (int i = 0; i < T; i++) {
        double s = 0.0;
        for (int k = 0; k < T; k++) s += Minv[i * T + k] * yh[(size_t)k * n];
        rhs[i] = sn * s;
        for (int k = 0; k < T; k++) N0[i * T + k] = (double)n * Minv[i * T + k];
      }
      if (sb_chol(N0, T)) {
        free(lam);
        free(yh);
        return 1;
      }
      sb_chol_solve(N0, T, rhs);
      for (int t = 0; t < T; t++) tau_hat[t] = rhs[t];
    } else {
      for (int t = 0; t < T; t++) tau_hat[t] = tau_in[t];
    }
    (void)b;
  }
  /* per-frequency factorisation, in fixed blocks of frequencies whose sums
   * are added in order afterwards */
  const int64_t blk = 4096;
  const int64_t nblk = (n + blk - 1) / blk;
  long double* pq = (long double*)calloc((size_t)nblk, sizeof(long double));
  long double* pl = (long double*)calloc((size_t)nblk, sizeof(long double));
  int bad = 0;
  if (!pq || !pl) {
    free(pq);
    free(pl);
    free(lam);
    free(yh);
    return 3;
  }
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
  for (int64_t bi = 0; bi < nblk; bi++) {
    long double sq = 0.0L, sl = 0.0L;
    const int64_t f1 = (bi + 1) * blk < n ? (bi + 1) * blk : n;
    for (int64_t f = bi * blk; f < f1; f++) {
      double A[SB_MAXT * SB_MAXT], r[SB_MAXT], a[SB_MAXT];
      for (int t = 0; t < T; t++)
        for (int u = 0; u <= t; u++)
          A[t * T + u] = R[t * T + u] * lam[(size_t)colof[t][u] * n + f] + (t == u ? xi[t] : 0.0);
      if (sb_chol(A, T)) {
        bad = 1;
        continue;
      }
      for (int t = 0; t < T; t++) {
        r[t] = yh[(size_t)t * n + f] - (f == 0 ? sn * tau_hat[t] : 0.0);
        a[t] = r[t];
        sl += 2.0L * logl((long double)A[t * T + t]);
      }
      sb_chol_solve(A, T, a);
      for (int t = 0; t < T; t++) {
        sq += (long double)r[t] * a[t];
        if (alpha) alpha[(size_t)t * n + f] = a[t];
      }
    }
    pq[bi] = sq;
    pl[bi] = sl;
  }
  long double q = 0.0L, l = 0.0L;
  for (int64_t bi = 0; bi < nblk; bi++) {
    q += pq[bi];
    l += pl[bi];
  }
  free(pq);
  free(pl);
  free(lam);
  free(yh);
  if (bad) return 1;
  out3[0] = (double)q;
  out3[1] = (double)l;
  out3[2] = (double)(q + l);
  if (alpha) {
    /* alpha_t = V ahat_t = H ahat_t / sqrt(n) */
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < T; t++) {
      double* v = alpha + (size_t)t * n;
      sb_walsh(v, n);
      for (int64_t f = 0; f < n; f++) v[f] /= sn;
    }
  }
  return 0;
}

/* Posterior mean at M test digits xs[M][d]: mean[M][T] =
 * tau_t + sum_u R_tu sum_k Q(xs XOR x_uk) alpha_uk over the T equal-size
 * tasks of n = 2^m points (alpha [T][n] from sb_mle_equal). */
int sb_mean(int T, int d, int m, const uint32_t* gen, const uint32_t* shift, int order,
            double gamma, const double* eta, const double* R, const double* tau,
            const double* alpha, int64_t M, const uint32_t* xs, double* mean) {
  if (T < 1 || T > SB_MAXT || d < 1 || d > 64 || m < 0 || m > 30) return 2;
  const int64_t n = (int64_t)1 << m;
  uint32_t* z = (uint32_t*)malloc((size_t)n * d * sizeof(uint32_t));
  if (!z) return 3;
  sb_points(gen, d, n, z);
  for (int64_t k = 0; k < M; k++) {
    long double s[SB_MAXT];
    for (int u = 0; u < T; u++) {
      long double acc = 0.0L;
#pragma omp parallel for schedule(static) reduction(+ : acc)
      for (int64_t i = 0; i < n; i++) {
        uint32_t a[64];
        for (int j = 0; j < d; j++) a[j] = xs[k * d + j] ^ z[i * d + j] ^ shift[u * d + j];
        acc += (long double)sb_q(d, order, gamma, eta, a) * alpha[(size_t)u * n + i];
      }
      s[u] = acc;
    }
    for (int t = 0; t < T; t++) {
      long double v = tau[t];
      for (int u = 0; u < T; u++) v += (long double)R[t * T + u] * s[u];
      mean[k * T + t] = (double)v;
    }
  }
  free(z);
  return 0;
}

/* Correlated sine targets (the synthetic target family of the benchmark
 * workloads) at the points of T equal-size net tasks, plus given noise:
 *   y_t(x) = rho_t g_0(x) + sqrt(1 - rho_t^2) g_{t+1}(x) + noise_t,
 *   g_k(x) = sum_j sin(2 pi freq[k][j] x_j + phase[k][j]) / (j + 1),
 * freq and phase [T+1][d], y [T][n]. */
int sb_targets_corr_sines(int T, int d, int m, const uint32_t* gen, const uint32_t* shift,
                          const double* freq, const double* phase, const double* rho,
                          const double* noise, double* y) {
  if (T < 1 || T > SB_MAXT || d < 1 || d > 64 || m < 0 || m > 30) return 2;
  const int64_t n = (int64_t)1 << m;
  uint32_t* z = (uint32_t*)malloc((size_t)n * d * sizeof(uint32_t));
  if (!z) return 3;
  sb_points(gen, d, n, z);
  const double tp = 2.0 * M_PI;
  for (int t = 0; t < T; t++) {
    const double a = rho[t], b = sqrt(1.0 - rho[t] * rho[t]);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
      double g0 = 0.0, g1 = 0.0;
      for (int j = 0; j < d; j++) {
        const double x = (double)(z[i * d + j] ^ shift[t * d + j]) * 0x1p-32;
        g0 += sin(tp * freq[j] * x + phase[j]) / (j + 1);
        g1 += sin(tp * freq[(t + 1) * d + j] * x + phase[(t + 1) * d + j]) / (j + 1);
      }
      y[(size_t)t * n + i] = a * g0 + b * g1 + noise[(size_t)t * n + i];
    }
  }
  free(z);
  return 0;
}

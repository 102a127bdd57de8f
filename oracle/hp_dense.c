/*
 * Extended-precision twin of the dense oracle (test infrastructure only).
 *
 * Same definitions as oracle/dense.py, written out in plain C loops in
 * `real` = long double (default build) or __float128 (-DORACLE_QUAD):
 *   - Gram blocks  Ktilde_tt'[i,k] = R_tt' Q(x_ti, x_t'k) + delta xi_t
 *     (Section "Multitask Setting"; Eq. mtprod; Eq. prod_kernel),
 *   - Cholesky, log det Ktilde = 2 sum log L_ii,
 *   - optimal means (E K^-1 E^T) tau = E K^-1 y (Eq. MTGP_optimal_tau),
 *   - quad = r^T K^-1 r, r = y - E^T tau (Eq. MTGP_MLE_GCV_loss),
 *   - posterior mean tau_t + sum_t' R_tt' sum_k Q(x*, x_t'k) alpha_t'k
 *     (Eq. MTGP_post_mean_cov).
 * Kernels: DSI orders 1..4 (Eq. DSI_kernel_1d_ex; order 1 read as
 * 1 - 3 t_1, the zero-mean order-one Walsh kernel) and SI orders 1..3
 * (Eq. SI_kernel_1d_ex).  Digits u stand for x = u 2^-32 (exact here).
 * Nothing here is shared with, or called by, the GPU library.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#ifdef ORACLE_QUAD
#include <quadmath.h>
typedef __float128 real;
#define RLOG logq
#define RSQRT sqrtq
#define RLDEXP ldexpq
static const real RPI = M_PIq;
#define HP_EXPORT(name) name##_quad
#else
typedef long double real;
#define RLOG logl
#define RSQRT sqrtl
#define RLDEXP ldexpl
static const real RPI = 3.141592653589793238462643383279502884L;
#define HP_EXPORT(name) name##_ld
#endif

/* beta(x) = -floor(log2 x), beta(0) = 0, for x = u 2^-32 */
static int beta_of(uint32_t u) {
  if (u == 0) return 0;
  int hb = 31;
  while (!((u >> hb) & 1u)) hb--;
  return 32 - hb;
}

static real t_nu(uint32_t u, int nu) {
  if (u == 0) return (real)0;
  return RLDEXP((real)1, -nu * beta_of(u));
}

static real dsi_khat(int alpha, uint32_t u) {
  real x = RLDEXP((real)u, -32);
  real b = (real)beta_of(u);
  real t1 = t_nu(u, 1), t2 = t_nu(u, 2), t3 = t_nu(u, 3);
  switch (alpha) {
    case 1: return (real)6 * ((real)1 / 6 - t1 / 2);
    case 2: return -1 - b * x + (real)5 / 2 * (1 - t1);
    case 3: return -1 + b * x * x - 5 * (1 - t1) * x + (real)43 / 18 * (1 - t2);
    case 4: {
      /* digits beyond the 32nd are zero: tail sum_{a>32} 8^-(a-1) = (8/7) 8^-32 */
      real s = 0;
      for (int a = 1; a <= 32; a++) {
        int xa = (u >> (32 - a)) & 1u;
        s += (1 - 2 * xa) * RLDEXP((real)1, -3 * (a - 1));
      }
      s += (real)8 / 7 * RLDEXP((real)1, -96);
      return -1 - (real)2 / 3 * b * x * x * x + 5 * (1 - t1) * x * x
             - (real)43 / 9 * (1 - t2) * x + (real)701 / 294 * (1 - t3)
             + b * (s / 48 - (real)1 / 42);
    }
  }
  return 0;
}

static real si_kern(int alpha, uint32_t u) {
  real x = RLDEXP((real)u, -32);
  real tp = 2 * RPI, c = 1, bp = 0;
  int p = 2 * alpha;
  for (int k = 0; k < p; k++) c *= tp;
  for (int k = 2; k <= p; k++) c /= k;
  if (!(alpha & 1)) c = -c;
  if (p == 2) bp = x * x - x + (real)1 / 6;
  else if (p == 4) bp = x * x * x * x - 2 * x * x * x + x * x - (real)1 / 30;
  else if (p == 6) bp = x * x * x * x * x * x - 3 * x * x * x * x * x + (real)5 / 2 * x * x * x * x
                        - x * x / 2 + (real)1 / 42;
  return c * bp;
}

typedef struct {
  int family, d, order, adaptive;
  real gamma, eta[64], b[4];
} kspec;

static real qkern(const kspec* k, const uint32_t* xa, const uint32_t* xb) {
  real q = k->gamma;
  for (int j = 0; j < k->d; j++) {
    uint32_t u = (k->family == 0) ? (xa[j] ^ xb[j]) : (uint32_t)(xa[j] - xb[j]);
    real kv = 0;
    if (k->family == 0) {
      if (k->adaptive) {
        for (int a = 1; a <= 4; a++) kv += k->b[a - 1] * dsi_khat(a, u);
      } else {
        kv = dsi_khat(k->order, u);
      }
    } else {
      kv = si_kern(k->order, u);
    }
    q *= 1 + k->eta[j] * kv;
  }
  return q;
}

/* Solve L L^T x = b in place (L lower, row-major). */
static void chol_solve(const real* L, int N, real* x) {
  for (int i = 0; i < N; i++) {
    real s = x[i];
    for (int k = 0; k < i; k++) s -= L[(size_t)i * N + k] * x[k];
    x[i] = s / L[(size_t)i * N + i];
  }
  for (int i = N - 1; i >= 0; i--) {
    real s = x[i];
    for (int k = i + 1; k < N; k++) s -= L[(size_t)k * N + i] * x[k];
    x[i] = s / L[(size_t)i * N + i];
  }
}

/*
 * Returns 0 on success, -1 if Ktilde is not positive definite, -2 on a bad
 * argument or allocation failure.  X: [N][d] digits, task-major; y: [N];
 * B: [T][s]; out[0] = quad, out[1] = logdet, out[2] = quad + logdet; tau_hat: [T]; Xs: [M][d];
 * mean: [M][T] (may be NULL when M == 0).
 */
int HP_EXPORT(hp_mtgp)(int family, int T, int d, const int* n, const uint32_t* X,
                       int order, int adaptive, const double* b, double gamma,
                       const double* eta, const double* xi, int s, const double* B,
                       const double* zeta, int profile, const double* tau_in,
                       const double* y, double* out, double* tau_hat, int M,
                       const uint32_t* Xs, double* mean) {
  if (T < 1 || T > 64 || d < 1 || d > 64) return -2;
  kspec ks;
  ks.family = family; ks.d = d; ks.order = order; ks.adaptive = adaptive;
  ks.gamma = gamma;
  for (int j = 0; j < d; j++) ks.eta[j] = eta[j];
  for (int a = 0; a < 4; a++) ks.b[a] = adaptive ? b[a] : 0;
  real R[64 * 64];
  for (int t = 0; t < T; t++)
    for (int u = 0; u < T; u++) {
      real acc = (t == u) ? (real)zeta[t] : 0;
      for (int k = 0; k < s; k++) acc += (real)B[t * s + k] * (real)B[u * s + k];
      R[t * T + u] = acc;
    }
  int off[65];
  off[0] = 0;
  for (int t = 0; t < T; t++) off[t + 1] = off[t] + n[t];
  int N = off[T];
  real* K = (real*)malloc(sizeof(real) * (size_t)N * N);
  real* v = (real*)malloc(sizeof(real) * (size_t)N * (T + 2));
  if (!K || !v) { free(K); free(v); return -2; }
  for (int t = 0; t < T; t++)
    for (int i = off[t]; i < off[t + 1]; i++)
      for (int u = 0; u < T; u++)
        for (int k = off[u]; k < off[u + 1]; k++) {
          real q = R[t * T + u] * qkern(&ks, X + (size_t)i * d, X + (size_t)k * d);
          if (i == k) q += (real)xi[t];
          K[(size_t)i * N + k] = q;
        }
  /* Cholesky, lower triangle in place */
  for (int j = 0; j < N; j++) {
    real dsum = K[(size_t)j * N + j];
    for (int k = 0; k < j; k++) dsum -= K[(size_t)j * N + k] * K[(size_t)j * N + k];
    if (!(dsum > 0)) { free(K); free(v); return -1; }
    real ljj = RSQRT(dsum);
    K[(size_t)j * N + j] = ljj;
    for (int i = j + 1; i < N; i++) {
      real a = K[(size_t)i * N + j];
      for (int k = 0; k < j; k++) a -= K[(size_t)i * N + k] * K[(size_t)j * N + k];
      K[(size_t)i * N + j] = a / ljj;
    }
  }
  real logdet = 0;
  for (int j = 0; j < N; j++) logdet += 2 * RLOG(K[(size_t)j * N + j]);
  real tau[64];
  if (profile) {
    /* columns: K^-1 E^T (T of them) and K^-1 y */
    for (int c = 0; c <= T; c++) {
      real* col = v + (size_t)c * N;
      for (int i = 0; i < N; i++) col[i] = 0;
      if (c < T) for (int i = off[c]; i < off[c + 1]; i++) col[i] = 1;
      else for (int i = 0; i < N; i++) col[i] = y[i];
      chol_solve(K, N, col);
    }
    real Pi[64 * 65];
    for (int t = 0; t < T; t++) {
      for (int u = 0; u <= T; u++) {
        real acc = 0;
        for (int i = off[t]; i < off[t + 1]; i++) acc += v[(size_t)u * N + i];
        Pi[t * (T + 1) + u] = acc;   /* [Pi | E K^-1 y] augmented */
      }
    }
    /* Gaussian elimination with partial pivoting on the T x T system */
    for (int c = 0; c < T; c++) {
      int p = c;
      for (int r = c + 1; r < T; r++) {
        real a = Pi[r * (T + 1) + c], bb = Pi[p * (T + 1) + c];
        if ((a < 0 ? -a : a) > (bb < 0 ? -bb : bb)) p = r;
      }
      for (int k = 0; k <= T; k++) {
        real tmp = Pi[c * (T + 1) + k];
        Pi[c * (T + 1) + k] = Pi[p * (T + 1) + k];
        Pi[p * (T + 1) + k] = tmp;
      }
      for (int r = c + 1; r < T; r++) {
        real f = Pi[r * (T + 1) + c] / Pi[c * (T + 1) + c];
        for (int k = c; k <= T; k++) Pi[r * (T + 1) + k] -= f * Pi[c * (T + 1) + k];
      }
    }
    for (int c = T - 1; c >= 0; c--) {
      real acc = Pi[c * (T + 1) + T];
      for (int k = c + 1; k < T; k++) acc -= Pi[c * (T + 1) + k] * tau[k];
      tau[c] = acc / Pi[c * (T + 1) + c];
    }
  } else {
    for (int t = 0; t < T; t++) tau[t] = tau_in[t];
  }
  real* alpha = v + (size_t)(T + 1) * N;
  for (int t = 0; t < T; t++)
    for (int i = off[t]; i < off[t + 1]; i++) alpha[i] = (real)y[i] - tau[t];
  real* r = (real*)malloc(sizeof(real) * (size_t)N);
  if (!r) { free(K); free(v); return -2; }
  memcpy(r, alpha, sizeof(real) * (size_t)N);
  chol_solve(K, N, alpha);
  real quad = 0;
  for (int i = 0; i < N; i++) quad += r[i] * alpha[i];
  out[0] = (double)quad;
  out[1] = (double)logdet;
  out[2] = (double)(quad + logdet);
  for (int t = 0; t < T; t++) tau_hat[t] = (double)tau[t];
  for (int m = 0; m < M; m++) {
    real kv[64];
    for (int u = 0; u < T; u++) {
      real acc = 0;
      for (int k = off[u]; k < off[u + 1]; k++)
        acc += qkern(&ks, Xs + (size_t)m * d, X + (size_t)k * d) * alpha[k];
      kv[u] = acc;
    }
    for (int t = 0; t < T; t++) {
      real acc = tau[t];
      for (int u = 0; u < T; u++) acc += R[t * T + u] * kv[u];
      mean[(size_t)m * T + t] = (double)acc;
    }
  }
  free(r);
  free(K);
  free(v);
  return 0;
}

/*
 * Extended-precision spectral route for digital nets of nested sizes
 * n_t = 2^m_t (test infrastructure only): the steps of the float64 spectral
 * oracle's MLE, in `real` arithmetic, for sizes the dense twin cannot factor.
 *   - Theorem "Fast MTGP computations" with the nested-size structure: for
 *     the pair (t, u) with n_t >= n_u (ties: t <= u), c_tu[i] =
 *     Q(z_i XOR Delta_t XOR Delta_u), i < n_t, and lambda_tu = H c_tu, the
 *     unnormalised Sylvester-ordered Walsh-Hadamard transform;
 *   - yhat_t = H y_t / sqrt(n_t);
 *   - frequencies fall into residue classes r < n_min; class r has members
 *     (t, k), k < n_t / n_min, at frequency r + n_min k, and its block
 *     M_r[(t, k), (u, k mod (n_u / n_min))] = sqrt(n_u / n_t) R_tu
 *     lambda_tu(r + n_min k) (and its transpose), plus xi_t on the diagonal;
 *   - profiled means from class 0 (Eq. MTGP_optimal_tau): with A[(t, 0), t]
 *     = sqrt(n_t), (A^T M_0^-1 A) tau = A^T M_0^-1 yhat(0);
 *   - L = sum_r rhat_r^T M_r^-1 rhat_r + log det M_r (Eq. MTGP_MLE_GCV_loss),
 *     rhat_r = yhat_r - [r = 0] A tau, by Cholesky.
 * z: [n_max][d] unshifted digits (z_i of the oracle's point generator),
 * shift: [T][d], y: task-major in the oracle's point order.  Classes run on
 * OpenMP threads; each accumulates its quad and log det in `real`.
 * Returns 0, -1 (a class block not positive definite) or -2 (bad argument or
 * allocation failure).
 */
static void hp_walsh(real* x, int64_t n) {
  for (int64_t h = 1; h < n; h <<= 1)
    for (int64_t i = 0; i < n; i += 2 * h)
      for (int64_t k = i; k < i + h; k++) {
        const real a = x[k], b = x[k + h];
        x[k] = a + b;
        x[k + h] = a - b;
      }
}

/* Cholesky of the c x c block in place (lower, row-major); 0 or -1 */
static int hp_chol(real* M, int c) {
  for (int j = 0; j < c; j++) {
    real dsum = M[(size_t)j * c + j];
    for (int k = 0; k < j; k++) dsum -= M[(size_t)j * c + k] * M[(size_t)j * c + k];
    if (!(dsum > 0)) return -1;
    const real ljj = RSQRT(dsum);
    M[(size_t)j * c + j] = ljj;
    for (int i = j + 1; i < c; i++) {
      real a = M[(size_t)i * c + j];
      for (int k = 0; k < j; k++) a -= M[(size_t)i * c + k] * M[(size_t)j * c + k];
      M[(size_t)i * c + j] = a / ljj;
    }
  }
  return 0;
}

int HP_EXPORT(hp_spectral_nets)(int T, int d, const int* m, const uint32_t* z,
                                const uint32_t* shift, int order, int adaptive, const double* b,
                                double gamma, const double* eta, const double* xi, int s,
                                const double* B, const double* zeta, int profile,
                                const double* tau_in, const double* y, double* out,
                                double* tau_hat) {
  if (T < 1 || T > 64 || d < 1 || d > 64) return -2;
  kspec ks;
  ks.family = 0; ks.d = d; ks.order = order; ks.adaptive = adaptive;
  ks.gamma = gamma;
  for (int j = 0; j < d; j++) ks.eta[j] = eta[j];
  for (int a = 0; a < 4; a++) ks.b[a] = adaptive ? b[a] : 0;
  real R[64 * 64];
  for (int t = 0; t < T; t++)
    for (int u = 0; u < T; u++) {
      real acc = (t == u) ? (real)zeta[t] : 0;
      for (int k = 0; k < s; k++) acc += (real)B[t * s + k] * (real)B[u * s + k];
      R[t * T + u] = acc;
    }
  int64_t n[64], yoff[65], nmin = INT64_MAX;
  int size[64], off[65];
  yoff[0] = 0;
  for (int t = 0; t < T; t++) {
    n[t] = (int64_t)1 << m[t];
    yoff[t + 1] = yoff[t] + n[t];
    if (n[t] < nmin) nmin = n[t];
  }
  off[0] = 0;
  for (int t = 0; t < T; t++) {
    size[t] = (int)(n[t] / nmin);
    off[t + 1] = off[t] + size[t];
  }
  const int c = off[T];
  /* spectra of the columns and of the data */
  real* lam[64 * 64] = {0};
  real* yh = (real*)malloc(sizeof(real) * (size_t)yoff[T]);
  int rc = yh ? 0 : -2;
  for (int t = 0; t < T && !rc; t++)
    for (int u = 0; u < T && !rc; u++) {
      if (!(n[t] > n[u] || (n[t] == n[u] && t <= u))) continue;
      real* col = (real*)malloc(sizeof(real) * (size_t)n[t]);
      if (!col) { rc = -2; break; }
      uint32_t dsh[64];
      for (int j = 0; j < d; j++) dsh[j] = shift[t * d + j] ^ shift[u * d + j];
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n[t]; i++) col[i] = qkern(&ks, z + (size_t)i * d, dsh);
      hp_walsh(col, n[t]);
      lam[t * T + u] = col;
    }
  for (int t = 0; t < T && !rc; t++) {
    real* v = yh + yoff[t];
    for (int64_t i = 0; i < n[t]; i++) v[i] = (real)y[yoff[t] + i];
    hp_walsh(v, n[t]);
    const real sc = 1 / RSQRT((real)n[t]);
    for (int64_t i = 0; i < n[t]; i++) v[i] *= sc;
  }
  real tau[64];
  real quad = 0, logdet = 0;
  if (!rc) {
    /* class 0: profiled means */
    real* M0 = (real*)malloc(sizeof(real) * (size_t)c * c);
    real* X = (real*)malloc(sizeof(real) * (size_t)c * (T + 1));
    if (!M0 || !X) rc = -2;
    if (!rc) {
      memset(M0, 0, sizeof(real) * (size_t)c * c);
      for (int t = 0; t < T; t++)
        for (int u = 0; u < T; u++) {
          const real* L = lam[t * T + u];
          if (!L) continue;
          const real f = RSQRT((real)n[u] / (real)n[t]) * R[t * T + u];
          for (int k = 0; k < size[t]; k++) {
            const int l = k % size[u];
            const real v = f * L[(int64_t)nmin * k];
            M0[(size_t)(off[t] + k) * c + off[u] + l] += v;
            if (t != u) M0[(size_t)(off[u] + l) * c + off[t] + k] += v;
          }
        }
      for (int t = 0; t < T; t++)
        for (int k = 0; k < size[t]; k++) M0[(size_t)(off[t] + k) * c + off[t] + k] += (real)xi[t];
      if (hp_chol(M0, c)) rc = -1;
    }
    if (!rc) {
      for (int q = 0; q <= T; q++) {
        real* col = X + (size_t)q * c;
        for (int i = 0; i < c; i++) col[i] = 0;
        if (q < T) col[off[q]] = RSQRT((real)n[q]);
        else
          for (int t = 0; t < T; t++)
            for (int k = 0; k < size[t]; k++) col[off[t] + k] = yh[yoff[t] + (int64_t)nmin * k];
        chol_solve(M0, c, col);
      }
      real G[64 * 65];
      for (int t = 0; t < T; t++)
        for (int q = 0; q <= T; q++) G[t * (T + 1) + q] = RSQRT((real)n[t]) * X[(size_t)q * c + off[t]];
      for (int cc = 0; cc < T; cc++) {
        int p = cc;
        for (int r = cc + 1; r < T; r++) {
          real a = G[r * (T + 1) + cc], bb = G[p * (T + 1) + cc];
          if ((a < 0 ? -a : a) > (bb < 0 ? -bb : bb)) p = r;
        }
        for (int k = 0; k <= T; k++) {
          real tmp = G[cc * (T + 1) + k];
          G[cc * (T + 1) + k] = G[p * (T + 1) + k];
          G[p * (T + 1) + k] = tmp;
        }
        for (int r = cc + 1; r < T; r++) {
          real f = G[r * (T + 1) + cc] / G[cc * (T + 1) + cc];
          for (int k = cc; k <= T; k++) G[r * (T + 1) + k] -= f * G[cc * (T + 1) + k];
        }
      }
      for (int cc = T - 1; cc >= 0; cc--) {
        real acc = G[cc * (T + 1) + T];
        for (int k = cc + 1; k < T; k++) acc -= G[cc * (T + 1) + k] * tau[k];
        tau[cc] = acc / G[cc * (T + 1) + cc];
      }
      if (!profile)
        for (int t = 0; t < T; t++) tau[t] = tau_in[t];
    }
    free(M0);
    free(X);
  }
  if (!rc) {
    int bad = 0;
#pragma omp parallel
    {
      real* M = (real*)malloc(sizeof(real) * (size_t)c * c);
      real* rh = (real*)malloc(sizeof(real) * (size_t)c);
      real q_loc = 0, ld_loc = 0;
      int bad_loc = (!M || !rh) ? -2 : 0;
#pragma omp for schedule(dynamic, 4)
      for (int64_t r = 0; r < nmin; r++) {
        if (bad_loc) continue;
        memset(M, 0, sizeof(real) * (size_t)c * c);
        for (int t = 0; t < T; t++)
          for (int u = 0; u < T; u++) {
            const real* L = lam[t * T + u];
            if (!L) continue;
            const real f = RSQRT((real)n[u] / (real)n[t]) * R[t * T + u];
            for (int k = 0; k < size[t]; k++) {
              const int l = k % size[u];
              const real v = f * L[r + (int64_t)nmin * k];
              M[(size_t)(off[t] + k) * c + off[u] + l] += v;
              if (t != u) M[(size_t)(off[u] + l) * c + off[t] + k] += v;
            }
          }
        for (int t = 0; t < T; t++)
          for (int k = 0; k < size[t]; k++) M[(size_t)(off[t] + k) * c + off[t] + k] += (real)xi[t];
        if (hp_chol(M, c)) { bad_loc = -1; continue; }
        for (int i = 0; i < c; i++) ld_loc += 2 * RLOG(M[(size_t)i * c + i]);
        for (int t = 0; t < T; t++)
          for (int k = 0; k < size[t]; k++) rh[off[t] + k] = yh[yoff[t] + r + (int64_t)nmin * k];
        if (r == 0)
          for (int t = 0; t < T; t++) rh[off[t]] -= RSQRT((real)n[t]) * tau[t];
        for (int i = 0; i < c; i++) {  /* forward substitution L z = rhat */
          real acc = rh[i];
          for (int k = 0; k < i; k++) acc -= M[(size_t)i * c + k] * rh[k];
          rh[i] = acc / M[(size_t)i * c + i];
          q_loc += rh[i] * rh[i];
        }
      }
#pragma omp critical
      {
        quad += q_loc;
        logdet += ld_loc;
        if (bad_loc && !bad) bad = bad_loc;
      }
      free(M);
      free(rh);
    }
    rc = bad;
  }
  for (int i = 0; i < T * T; i++) free(lam[i]);
  free(yh);
  if (rc) return rc;
  out[0] = (double)quad;
  out[1] = (double)logdet;
  out[2] = (double)(quad + logdet);
  for (int t = 0; t < T; t++) tau_hat[t] = (double)tau[t];
  return 0;
}

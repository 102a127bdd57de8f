// Device bodies of parameter decoding and of the final reductions / chain
// rule, shared by the per-plan kernels (solve.hip) and the many-fit kernels
// (batch.hip).
#pragma once
#include "kernels.h"

namespace mtgp {

// theta -> Params (thread 0 of the calling block), status cleared
__device__ inline void prep_device(const double* __restrict__ theta, Params* __restrict__ P,
                            const KDesc& kd, int* __restrict__ status) {
  if (threadIdx.x != 0) return;
  const int T = kd.T, d = kd.d, s = kd.s;
  const int nb = kd.adaptive ? 4 : 0;
  int o = 0;
  for (int t = 0; t < T; t++) P->tau[t] = theta[o + t];
  o += T;
  P->gamma = exp(theta[o]);
  o += 1;
  for (int j = 0; j < MTGP_MAXD; j++) P->eta[j] = j < d ? exp(theta[o + j]) : 0.0;
  o += d;
  for (int a = 0; a < 4; a++) P->b[a] = a < nb ? exp(theta[o + a]) : 0.0;
  o += nb;
  for (int t = 0; t < T; t++) P->xi[t] = exp(theta[o + t]);
  o += T;
  for (int i = 0; i < T * s; i++) P->B[i] = theta[o + i];
  o += T * s;
  for (int t = 0; t < T; t++) P->zeta[t] = exp(theta[o + t]);
  for (int t = 0; t < T; t++)
    for (int u = 0; u < T; u++) {
      double acc = (t == u) ? P->zeta[t] : 0.0;
      for (int k = 0; k < s; k++) acc += P->B[t * s + k] * P->B[u * s + k];
      P->R[t * MTGP_MAXT + u] = acc;
    }
  P->gamma_f = (float)P->gamma;
  for (int j = 0; j < MTGP_MAXD; j++) P->eta_f[j] = (float)P->eta[j];
  for (int a = 0; a < 4; a++) P->b_f[a] = (float)P->b[a];
  status[0] = 0;
  status[1] = 0;
  *reinterpret_cast<unsigned long long*>(status + 2) = ~0ull;
}

// The whole calling block (256 threads) takes part; thread 0 writes out3,
// tau_hat and grad.
__device__ inline void finalize_device(const double* __restrict__ sp, int nsolve,
                                const double* __restrict__ cs, const ColInfo* __restrict__ ci,
                                int ncol, const double* __restrict__ lp, int nld,
                                const double* __restrict__ yhat, int64_t n,
                                Params* __restrict__ P, const KDesc& kd,
                                double* __restrict__ out3, double* __restrict__ grad,
                                double* __restrict__ tau_hat) {
  __shared__ double red[16];
  __shared__ double sums[64];
  __shared__ double Gm[MTGP_MAXT * MTGP_MAXT];
  // the small tables of the chain rule, staged by all threads: the serial
  // code below then reads LDS instead of a chain of dependent global loads
  // (column pair -> R entry), about two memory latencies per column
  __shared__ double s_cs[MTGP_MAXCOL * (MTGP_MAXD + 5)];
  __shared__ int s_tu[2 * MTGP_MAXCOL];
  __shared__ double s_R[MTGP_MAXT * MTGP_MAXT];
  __shared__ double s_B[MTGP_MAXT * MTGP_MAXS];
  const int T = kd.T, d = kd.d, s = kd.s;
  const int ns = solve_ns(T);
  const int nq = adj_nq(d);
  if (grad) {
    for (int i = threadIdx.x; i < ncol * nq; i += blockDim.x) s_cs[i] = cs[i];
    for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
      s_tu[2 * c] = ci[c].t;
      s_tu[2 * c + 1] = ci[c].u;
    }
    for (int i = threadIdx.x; i < T * s; i += blockDim.x) s_B[i] = P->B[i];
  }
  for (int i = threadIdx.x; i < MTGP_MAXT * MTGP_MAXT; i += blockDim.x) s_R[i] = P->R[i];
  // all ns slots in one pass (fixed order): thread (g, q) sums the rows
  // g, g + ng, ... of slot q, then one thread per slot adds the ng groups
  __shared__ double part[256];
  const int ng = blockDim.x / ns;  // ns <= 2 + 3 MTGP_MAXT, so ng >= 5
  if ((int)threadIdx.x < ng * ns) {
    const int q = threadIdx.x % ns, g = threadIdx.x / ns;
    double v = 0.0;
    for (int b = g; b < nsolve; b += ng) v += sp[(size_t)b * ns + q];
    part[threadIdx.x] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < ns) {
    double v = 0.0;
    for (int g = 0; g < ng; g++) v += part[g * ns + threadIdx.x];
    sums[threadIdx.x] = v;
  }
  double ldx = 0.0;  // log pivots of the elimination stages (unequal sizes)
  if (lp)
    for (int b = threadIdx.x; b < nld; b += blockDim.x) ldx += lp[b];
  ldx = block_sum(ldx, red);
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (kd.gcv) {
    // GCV: sums[0] = q = r^T Ktilde^-2 r, sums[1] = s = tr Ktilde^-1
    const double q = sums[0], s2 = sums[1];
    out3[0] = q;
    out3[1] = s2;
    out3[2] = q / (s2 * s2);
    P->gcv_q = q;
    P->gcv_s = s2;
  } else {
    const double quad = sums[0], logdet = sums[1] + ldx;
    out3[0] = quad;
    out3[1] = logdet;
    out3[2] = quad + logdet;
  }
  const double sqn = sqrt((double)n);
  const int TMp = solve_tm(T);
  const int qG = 2, qX = 2 + TMp, qA = 2 + 2 * TMp;
  for (int t = 0; t < T; t++) {
    const int64_t y0 = (int64_t)t * n * (kd.family == FAM_LAT ? 2 : 1);
    const double tu = kd.unequal ? P->tau_used[t] : (kd.profile ? yhat[y0] / sqn : P->tau[t]);
    P->tau_used[t] = tu;
    if (tau_hat) tau_hat[t] = tu;
  }
  if (!grad) return;
  // G_tu = sum_f Re(W_ut lambda_tu): diagonal from the solve, cross-task from
  // the pair columns (their w c sums are 2 G_tu); kernel-hyperparameter sums
  // of a pair column carry R_tu, diagonal columns carry it in their weights
  for (int t = 0; t < T; t++) Gm[t * MTGP_MAXT + t] = sums[qG + t];
  double geta[MTGP_MAXD + 4];
  for (int q = 0; q < d + 4; q++) geta[q] = 0.0;
  for (int c = 0; c < ncol; c++) {
    const int t = s_tu[2 * c], u = s_tu[2 * c + 1];
    const double* row = s_cs + (size_t)c * nq;
    const double Rc = t == u ? 1.0 : s_R[t * MTGP_MAXT + u];
    if (t != u) Gm[t * MTGP_MAXT + u] = Gm[u * MTGP_MAXT + t] = 0.5 * row[0];
    for (int q = 0; q < d + 4; q++) geta[q] += Rc * row[1 + q];
  }
  auto G = [&](int t, int u) { return Gm[t * MTGP_MAXT + u]; };
  int o = 0;
  for (int t = 0; t < T; t++)
    grad[o + t] = kd.profile ? 0.0 : -2.0 * sqrt(ldexp(1.0, kd.m[t])) * sums[qA + t];
  o += T;
  double gg = 0.0;
  for (int t = 0; t < T; t++)
    for (int u = 0; u < T; u++) gg += s_R[t * MTGP_MAXT + u] * G(t, u);
  grad[o++] = gg;
  for (int j = 0; j < d; j++) grad[o + j] = geta[j];
  o += d;
  if (kd.adaptive) {
    for (int a = 0; a < 4; a++) grad[o + a] = P->b[a] * geta[d + a];
    o += 4;
  }
  for (int t = 0; t < T; t++) grad[o + t] = P->xi[t] * sums[qX + t];
  o += T;
  for (int t = 0; t < T; t++)
    for (int k = 0; k < s; k++) {
      double acc = 0.0;
      for (int u = 0; u < T; u++) acc += 2.0 * G(t, u) * s_B[u * s + k];
      grad[o + t * s + k] = acc;
    }
  o += T * s;
  for (int t = 0; t < T; t++) grad[o + t] = P->zeta[t] * G(t, t);
}

}  // namespace mtgp

// Multitask Bayesian cubature (Section "Extensions for Bayesian Cubature",
// the multitask theorem): the posterior of the task integrals
// mu_t = int f(t, x) dx is N(mu_hat, Sigma) with
//   mu_hat = tau + gamma R E Ktilde^-1 (y - E^T tau),
//   Sigma  = gamma R - gamma^2 R Pi R,   Pi = E Ktilde^-1 E^T,
// gamma = int Q(x, x') dx' being the kernel's gamma (the univariate DSI and
// SI kernels integrate to 0).  In the transformed basis only frequency 0 of
// every task enters (V^dagger 1 = sqrt(n) e_0):
//   Pi_tu = sqrt(n_t n_u) (Lambda^-1)_{(t,0),(u,0)},
//   (E Ktilde^-1 r)_t = sqrt(n_t) ahat_t(0).
// Equal sizes: Lambda(0) is the T x T block of frequency 0, inverted here;
// nested sizes: the elimination leaves Pi in the parameter block.  O(T^3).
#include "kernels.h"

namespace mtgp {

template <typename SR>
__global__ void cubature_kernel(const SR* __restrict__ cols, CubDesc cd,
                                const double* __restrict__ ahat, const Params* __restrict__ P,
                                KDesc kd, double* __restrict__ mu, double* __restrict__ Sigma) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int T = kd.T;
  const int cpl = kd.family == FAM_LAT ? 2 : 1;
  double Pi[MTGP_MAXT][MTGP_MAXT];
  if (cd.equal) {
    // Lambda(0)_tu = R_tu lambda_p(0) + delta_tu xi_t (real at f = 0)
    double A[MTGP_MAXT][2 * MTGP_MAXT];
    for (int t = 0; t < T; t++)
      for (int u = 0; u < T; u++) {
        const int c = cd.pair_col[t < u ? t : u][t < u ? u : t];
        const double lam = (double)cols[(size_t)c * cd.n * cpl];
        A[t][u] = P->R[t * MTGP_MAXT + u] * lam + (t == u ? P->xi[t] : 0.0);
        A[t][T + u] = t == u ? 1.0 : 0.0;
      }
    // Gauss-Jordan with partial pivoting (T <= 16, FP64)
    for (int c = 0; c < T; c++) {
      int pv = c;
      for (int i = c + 1; i < T; i++)
        if (fabs(A[i][c]) > fabs(A[pv][c])) pv = i;
      for (int k = 0; k < 2 * T; k++) {
        const double tmp = A[c][k];
        A[c][k] = A[pv][k];
        A[pv][k] = tmp;
      }
      const double inv = 1.0 / A[c][c];
      for (int k = 0; k < 2 * T; k++) A[c][k] *= inv;
      for (int i = 0; i < T; i++) {
        if (i == c) continue;
        const double fct = A[i][c];
        for (int k = 0; k < 2 * T; k++) A[i][k] -= fct * A[c][k];
      }
    }
    for (int t = 0; t < T; t++)
      for (int u = 0; u < T; u++) Pi[t][u] = (double)cd.n * A[t][T + u];
  } else {
    for (int t = 0; t < T; t++)
      for (int u = 0; u < T; u++) Pi[t][u] = P->Pi[t * MTGP_MAXT + u];
  }
  double Ea[MTGP_MAXT];
  for (int t = 0; t < T; t++)
    Ea[t] = sqrt(ldexp(1.0, kd.m[t])) * ahat[(size_t)cd.task_off[t] * cpl];
  const double g = P->gamma;
  double RP[MTGP_MAXT][MTGP_MAXT];
  for (int t = 0; t < T; t++) {
    double s = 0.0;
    for (int u = 0; u < T; u++) s += P->R[t * MTGP_MAXT + u] * Ea[u];
    mu[t] = P->tau_used[t] + g * s;
    for (int u = 0; u < T; u++) {
      double v = 0.0;
      for (int k = 0; k < T; k++) v += P->R[t * MTGP_MAXT + k] * Pi[k][u];
      RP[t][u] = v;
    }
  }
  for (int t = 0; t < T; t++)
    for (int u = 0; u < T; u++) {
      double v = 0.0;
      for (int k = 0; k < T; k++) v += RP[t][k] * P->R[k * MTGP_MAXT + u];
      Sigma[t * T + u] = g * P->R[t * MTGP_MAXT + u] - g * g * v;
    }
}

template <typename SR>
int launch_cubature(const SR* cols, const CubDesc& cd, const double* ahat, const Params* P,
                    const KDesc& kd, double* mu, double* Sigma, hipStream_t st) {
  hipLaunchKernelGGL((cubature_kernel<SR>), dim3(1), dim3(64), 0, st, cols, cd, ahat, P, kd, mu,
                     Sigma);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_cubature<double>(const double*, const CubDesc&, const double*, const Params*,
                                     const KDesc&, double*, double*, hipStream_t);
template int launch_cubature<float>(const float*, const CubDesc&, const double*, const Params*,
                                    const KDesc&, double*, double*, hipStream_t);

}  // namespace mtgp

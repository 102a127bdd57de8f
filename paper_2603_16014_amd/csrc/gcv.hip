// GCV loss of the multitask GP (Eq. MTGP_MLE_GCV_loss),
//   L_GCV = r^T Ktilde^-2 r / tr^2(Ktilde^-1),  r = y - E^T tau,
// on the equal-size spectral factorisation Ktilde = V Lambda V^dagger:
//   q = r^T Ktilde^-2 r = sum_f |ahat(f)|^2,  ahat = Lambda(f)^-1 rhat(f),
//   s = tr Ktilde^-1    = sum_f tr Lambda(f)^-1.
// With equal sizes the optimal GCV means (Eq. MTGP_optimal_tau) are the
// per-task sample means, as for the MLE, so rhat(0) = 0 when they are profiled.
//
// Gradient (the paper gives none; exact derivative): with bhat = Lambda^-1 ahat,
//   dL = sum_f tr(W(f) dLambda(f)),
//   W = -(bhat ahat^H + ahat bhat^H) / s^2 + (2 q / s^3) Lambda^-2,
// which feeds the same adjoint transform, derivative reduction and chain rule
// as the MLE loss; q and s come from a first pass (the loss).  With fixed
// means dL/dtau_t = -2 sqrt(n) Re bhat_t(0) / s^2; the pass stores
// Re bhat_t(0) / s^2 where the MLE stores ahat_t(0).
//
// One kernel for both families: digital nets in real arithmetic (S = double),
// lattices in complex arithmetic (S = zc, Hermitian Lambda).
#include "kernels.h"

namespace mtgp {

namespace {

struct zc {
  double x, y;
};
__device__ inline double re(double a) { return a; }
__device__ inline double re(zc a) { return a.x; }
__device__ inline double cj(double a) { return a; }
__device__ inline zc cj(zc a) { return {a.x, -a.y}; }
__device__ inline double mul(double a, double b) { return a * b; }
__device__ inline zc mul(zc a, zc b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline double add(double a, double b) { return a + b; }
__device__ inline zc add(zc a, zc b) { return {a.x + b.x, a.y + b.y}; }
__device__ inline double sub(double a, double b) { return a - b; }
__device__ inline zc sub(zc a, zc b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline double scl(double a, double s) { return a * s; }
__device__ inline zc scl(zc a, double s) { return {a.x * s, a.y * s}; }
__device__ inline double abs2(double a) { return a * a; }
__device__ inline double abs2(zc a) { return a.x * a.x + a.y * a.y; }
template <typename S> __device__ inline S zero();
template <> __device__ inline double zero<double>() { return 0.0; }
template <> __device__ inline zc zero<zc>() { return {0.0, 0.0}; }
template <typename S> __device__ inline S real_s(double v);
template <> __device__ inline double real_s<double>(double v) { return v; }
template <> __device__ inline zc real_s<zc>(double v) { return {v, 0.0}; }

template <int TM>
__device__ constexpr int pk(int i, int j) {
  return i * (i + 1) / 2 + j;
}

// value of column c at frequency f (interleaved complex for lattices)
template <typename S, typename SR>
__device__ inline S col_at(const SR* cols, int c, int64_t n, int64_t f);
template <>
__device__ inline double col_at<double, double>(const double* cols, int c, int64_t n, int64_t f) {
  return cols[(int64_t)c * n + f];
}
template <>
__device__ inline double col_at<double, float>(const float* cols, int c, int64_t n, int64_t f) {
  return (double)cols[(int64_t)c * n + f];
}
template <>
__device__ inline zc col_at<zc, double>(const double* cols, int c, int64_t n, int64_t f) {
  const size_t at = ((size_t)c * n + f) * 2;
  return {cols[at], cols[at + 1]};
}
template <>
__device__ inline zc col_at<zc, float>(const float* cols, int c, int64_t n, int64_t f) {
  const size_t at = ((size_t)c * n + f) * 2;
  return {(double)cols[at], (double)cols[at + 1]};
}
template <typename S, typename SR>
__device__ inline void col_put(SR* cols, int c, int64_t n, int64_t f, S v);
template <typename SR>
__device__ inline void col_put(SR* cols, int c, int64_t n, int64_t f, double v) {
  cols[(int64_t)c * n + f] = (SR)v;
}
template <typename SR>
__device__ inline void col_put(SR* cols, int c, int64_t n, int64_t f, zc v) {
  const size_t at = ((size_t)c * n + f) * 2;
  cols[at] = (SR)v.x;
  cols[at + 1] = (SR)v.y;
}

}  // namespace

template <typename S, typename SR, int TM, bool GRAD>
__global__ __launch_bounds__(256) void gcv_eq_kernel(SR* __restrict__ cols, int64_t n, PairMap pm,
                                                     const double* __restrict__ yhat,
                                                     const Params* __restrict__ P, KDesc kd,
                                                     double* __restrict__ partials,
                                                     int* __restrict__ status) {
  constexpr int NP = TM * (TM + 1) / 2;
  constexpr int NQ = 2 + 3 * TM;
  constexpr bool CPLX = sizeof(S) == 16;
  __shared__ double red[4 * NQ];
  const int T = kd.T;
  double vals[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) vals[q] = 0.0;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f < n) {
    S A[NP], r[TM];
    double lamd[TM];
#pragma unroll
    for (int i = 0; i < TM; i++) {
#pragma unroll
      for (int j = 0; j <= i; j++) {
        if (i < T) {
          S l = col_at<S, SR>(cols, pm.at(j, i), n, f);
          if (i == j) {
            l = real_s<S>(re(l));
            lamd[i] = re(l);
          }
          // lower entry (i, j): Lambda_ij = conj(Lambda_ji) = R_ji conj(lambda_ji)
          A[pk<TM>(i, j)] = add(scl(cj(l), P->R[j * MTGP_MAXT + i]),
                                real_s<S>(i == j ? P->xi[i] : 0.0));
        } else {
          if (i == j) lamd[i] = 0.0;
          A[pk<TM>(i, j)] = real_s<S>(i == j ? 1.0 : 0.0);
        }
      }
      if (i < T) {
        S yv;
        if constexpr (CPLX) yv = S{yhat[((size_t)i * n + f) * 2], yhat[((size_t)i * n + f) * 2 + 1]};
        else yv = real_s<S>(yhat[(size_t)i * n + f]);
        if (f == 0) yv = kd.profile ? zero<S>() : sub(yv, real_s<S>(sqrt((double)n) * P->tau[i]));
        r[i] = yv;
      } else {
        r[i] = zero<S>();
      }
    }
    // Lambda = L D L^H: strictly lower part of A becomes L
    double invD[TM], Dv[TM];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < TM; j++) {
      S u[TM];
      double dj = re(A[pk<TM>(j, j)]);
#pragma unroll
      for (int k = 0; k < j; k++) {
        const S l = A[pk<TM>(j, k)];
        u[k] = scl(l, Dv[k]);
        dj -= abs2(l) * Dv[k];
      }
      ok = ok && (dj > 0.0) && isfinite(dj);
      Dv[j] = dj;
      invD[j] = 1.0 / dj;
#pragma unroll
      for (int i = j + 1; i < TM; i++) {
        S v = A[pk<TM>(i, j)];
#pragma unroll
        for (int k = 0; k < j; k++) v = sub(v, mul(A[pk<TM>(i, k)], cj(u[k])));
        A[pk<TM>(i, j)] = scl(v, invD[j]);
      }
    }
    if (!ok) flag_bad(status, f);
    // ahat = Lambda^-1 rhat
    S a[TM];
#pragma unroll
    for (int i = 0; i < TM; i++) {
      S v = r[i];
#pragma unroll
      for (int k = 0; k < i; k++) v = sub(v, mul(A[pk<TM>(i, k)], a[k]));
      a[i] = v;
    }
#pragma unroll
    for (int i = TM - 1; i >= 0; i--) {
      S v = scl(a[i], invD[i]);
#pragma unroll
      for (int k = i + 1; k < TM; k++) v = sub(v, mul(cj(A[pk<TM>(k, i)]), a[k]));
      a[i] = v;
    }
    // X = L^-1 (unit lower) in place
#pragma unroll
    for (int i = 1; i < TM; i++) {
#pragma unroll
      for (int j = 0; j < i; j++) {
        S v = A[pk<TM>(i, j)];
#pragma unroll
        for (int k = j + 1; k < i; k++) v = add(v, mul(A[pk<TM>(i, k)], A[pk<TM>(k, j)]));
        A[pk<TM>(i, j)] = scl(v, -1.0);
      }
    }
    // Lambda^-1 (lower packed, Hermitian): (Lambda^-1)_ut = sum_{k >= u} conj(X_ku) X_kt / D_k for u >= t
    S AI[NP];
    double trace = 0.0;
#pragma unroll
    for (int u = 0; u < TM; u++) {
#pragma unroll
      for (int t = 0; t <= u; t++) {
        S v = t == u ? real_s<S>(invD[u]) : scl(A[pk<TM>(u, t)], invD[u]);
#pragma unroll
        for (int k = u + 1; k < TM; k++)
          v = add(v, scl(mul(cj(A[pk<TM>(k, u)]), A[pk<TM>(k, t)]), invD[k]));
        AI[pk<TM>(u, t)] = v;
      }
      if (u < T) trace += re(AI[pk<TM>(u, u)]);
    }
    double qf = 0.0;
#pragma unroll
    for (int t = 0; t < TM; t++)
      if (t < T) qf += abs2(a[t]);
    vals[0] += qf;
    vals[1] += trace;
    if (GRAD) {
      auto ai = [&](int i, int j) -> S {  // full Hermitian access
        return i >= j ? AI[pk<TM>(i, j)] : cj(AI[pk<TM>(j, i)]);
      };
      const double q = P->gcv_q, s = P->gcv_s;
      const double is2 = 1.0 / (s * s), c3 = 2.0 * q / (s * s * s);
      S b[TM];
#pragma unroll
      for (int t = 0; t < TM; t++) {
        S v = zero<S>();
#pragma unroll
        for (int u = 0; u < TM; u++) v = add(v, mul(ai(t, u), a[u]));
        b[t] = v;
      }
      if (f == 0) {
#pragma unroll
        for (int t = 0; t < TM; t++) vals[2 + 2 * TM + t] += re(b[t]) * is2;
      }
      double wdiag = 0.0;
#pragma unroll
      for (int u = 0; u < TM; u++) {
#pragma unroll
        for (int t = 0; t <= u; t++) {
          // W_tu = -(b_t conj(a_u) + a_t conj(b_u)) / s^2 + c3 (Lambda^-2)_tu
          S m2 = zero<S>();
#pragma unroll
          for (int k = 0; k < TM; k++) m2 = add(m2, mul(ai(t, k), ai(k, u)));
          const S w = add(scl(add(mul(b[t], cj(a[u])), mul(a[t], cj(b[u]))), -is2), scl(m2, c3));
          if (u < T) {
            if (t == u) {
              vals[2 + t] += re(w) * lamd[t];
              vals[2 + TM + t] += re(w);
              wdiag += P->R[t * MTGP_MAXT + t] * re(w);
            } else {
              col_put<SR>(cols, pm.at(t, u), n, f, scl(cj(w), 2.0));
            }
          }
        }
      }
      col_put<SR>(cols, pm.at(0, 0), n, f, real_s<S>(wdiag));
    }
  }
  block_sum_store<NQ>(vals, NQ, red, partials + (size_t)blockIdx.x * NQ);
}

template <typename SR>
int launch_gcv_eq(SR* cols, int64_t n, const PairMap& pm, const double* yhat, const Params* P,
                  const KDesc& kd, bool grad, double* partials, int* status, hipStream_t st) {
  const dim3 grid((unsigned)solve_blocks(n)), block(256);
#define MTGP_GCV(S, TMV)                                                                    \
  do {                                                                                      \
    if (grad)                                                                               \
      hipLaunchKernelGGL((gcv_eq_kernel<S, SR, TMV, true>), grid, block, 0, st, cols, n, pm, \
                         yhat, P, kd, partials, status);                                    \
    else                                                                                    \
      hipLaunchKernelGGL((gcv_eq_kernel<S, SR, TMV, false>), grid, block, 0, st, cols, n,   \
                         pm, yhat, P, kd, partials, status);                                \
  } while (0)
#define MTGP_GCV_T(S)                  \
  do {                                 \
    if (kd.T <= 1) MTGP_GCV(S, 1);     \
    else if (kd.T <= 2) MTGP_GCV(S, 2); \
    else if (kd.T <= 4) MTGP_GCV(S, 4); \
    else if (kd.T <= 8) MTGP_GCV(S, 8); \
    else MTGP_GCV(S, 16);              \
  } while (0)
  if (kd.family == FAM_LAT) MTGP_GCV_T(zc);
  else MTGP_GCV_T(double);
#undef MTGP_GCV_T
#undef MTGP_GCV
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_gcv_eq<double>(double*, int64_t, const PairMap&, const double*, const Params*,
                                   const KDesc&, bool, double*, int*, hipStream_t);
template int launch_gcv_eq<float>(float*, int64_t, const PairMap&, const double*, const Params*,
                                  const KDesc&, bool, double*, int*, hipStream_t);

}  // namespace mtgp

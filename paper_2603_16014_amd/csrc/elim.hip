// Nested unequal sample sizes without fill: Lambda = L D L^H in task order.
//
// Lambda couples node (t, f) only to the nodes (u, f mod n_u) of the other
// tasks (Theorem "Fast MTGP computations", item 3, tall case).  With tasks
// ordered by non-increasing size, the later neighbours of (t, f),
//   N(t, f) = {(u, f mod n_u) : u > t},
// are pairwise coupled themselves (n_v divides n_u), so eliminating the
// nodes in task order creates no fill: L has the pattern of Lambda.  This is
// the same elimination order as Algorithm "Inverse and log-determinant of
// Lambda" (the same pivots, hence the same log-determinant), kept sparse:
// O(N T^2) work and sum_t (T - t) n_t stored entries instead of dense blocks
// of size N / n_T.
//
// Pattern storage, complex (lattices) or real with zero imaginary part
// (digital sequences), all FP64: for a <= b and g < n_a,
//   S[so[a] + (b - a) n_a + g] = entry of row (b, g mod n_b), column (a, g).
// Right-looking factorisation: stage t updates, for u <= v later tasks,
//   S_uv[g] -= sum_{f < n_t, f = g mod n_u} S_tv[f] conj(S_tu[f]) / S_tt[f],
// and the forward substitution of the right-hand sides in the same way.
// The backward pass (tasks in reverse order) forms ahat = L^-H D^-1 z and,
// for the gradient, the entries of Z = Lambda^-1 on the pattern (the
// pattern is chordal, so they only need each other):
//   Z_{(u,.),(t,f)} = - sum_{v > t} Z_{(u,.),(v,.)} L_{(v,.),(t,f)},
//   Z_{(t,f),(t,f)} = 1 / d - sum_{u > t} conj(Z_{(u,.),(t,f)}) L_{(u,.),(t,f)},
// overwriting the factor column of (t, f) in place.
// Profiled means need the residue-0 entries of Lambda^-1 and Lambda^-1 yhat
// (Theorem "Fast MTGP computations", item 4): the T unit right-hand sides
// e_(u,0) are carried on the nodes of residue class 0 mod n_T only (the
// classes decouple), and ahat = Lambda^-1 yhat - sum_u sqrt(n_u) tau_u
// Lambda^-1 e_(u,0) is assembled in the final pass.
#include "kernels.h"
#include "elim_dev.h"

namespace mtgp {

template <typename SR>
__global__ void zf_init_kernel(const SR* __restrict__ cols, Alg1Desc A, const Params* __restrict__ P,
                               int family, int64_t N, const double* __restrict__ yhat,
                               z2* __restrict__ S, z2* __restrict__ rr, z2* __restrict__ U) {
  zf_init_body<SR>(cols, A, P, family, N, yhat, S, rr, U,
                   blockIdx.x * (int64_t)blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

__global__ __launch_bounds__(256) void zf_factor_kernel(Alg1Desc A, int t, int u, int G,
                                                        z2* __restrict__ S, z2* __restrict__ rr,
                                                        z2* __restrict__ U) {
  zf_factor_body(A, t, u, G, S, rr, U, blockIdx.x * (int64_t)blockDim.x + threadIdx.x,
                 (int64_t)gridDim.x * blockDim.x);
}

template <int TM, bool GRAD>
__global__ __launch_bounds__(256) void zf_back_kernel(Alg1Desc A, int t, z2* __restrict__ S,
                                                      z2* __restrict__ rr, z2* __restrict__ U,
                                                      double* __restrict__ logs,
                                                      int* __restrict__ status) {
  zf_back_body<TM, GRAD>(A, t, S, rr, U, logs, status,
                         blockIdx.x * (int64_t)blockDim.x + threadIdx.x,
                         (int64_t)gridDim.x * blockDim.x);
}

__global__ void zf_tau_kernel(Alg1Desc A, Params* P, const z2* __restrict__ rr,
                              const z2* __restrict__ U) {
  zf_tau_body(A, P, rr, U);
}

template <typename SR, int TM>
__global__ __launch_bounds__(256) void zf_final_kernel(SR* __restrict__ cols, Alg1Desc A, int64_t N,
                                                       const Params* __restrict__ P, int family,
                                                       int grad, const double* __restrict__ yhat,
                                                       const z2* __restrict__ S,
                                                       const z2* __restrict__ rr,
                                                       const z2* __restrict__ U,
                                                       double* __restrict__ ahat,
                                                       double* __restrict__ partials) {
  constexpr int NQ = 2 + 3 * TM;
  zf_final_body<SR, TM>(cols, A, N, P, family, grad, yhat, S, rr, U, ahat,
                        partials + (size_t)blockIdx.x * NQ,
                        blockIdx.x * (int64_t)blockDim.x + threadIdx.x,
                        (int64_t)gridDim.x * blockDim.x);
}

// GCV at nested sizes (Eq. MTGP_MLE_GCV_loss, Eq. MTGP_optimal_tau), loss
// only: q = |ahat|^2 with ahat = Lambda^-1 rhat, s = tr Lambda^-1 (the
// diagonal of the selected inverse), and the profiled means from
//   (E K^-2 E^T)_tu = sqrt(n_t n_u) (Lambda^-2)_{(t,0),(u,0)} = sqrt(n_t n_u) U_t^H U_u,
//   (E K^-2 y)_t = sqrt(n_t) (Lambda^-2 yhat)_{(t,0)} = sqrt(n_t) U_t^H (Lambda^-1 yhat),
// sums over residue class 0 (U_u = Lambda^-1 e_(u,0), supported there).
__global__ void zf_gcv_tau_kernel(Alg1Desc A, Params* P, const z2* __restrict__ rr,
                                  const z2* __restrict__ U) {
  __shared__ double M[MTGP_MAXT][MTGP_MAXT + 1];
  __shared__ double red[16];
  const int T = A.T;
  const int cs = A.m[T - 1];
  const int64_t ms = A.msz[T - 1];
  for (int e = 0; e < T * (T + 1); e++) {
    const int t = e / (T + 1), u = e - t * (T + 1);
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < ms; k += blockDim.x) {
      const z2 a = U[(int64_t)t * ms + k];
      z2 b;
      if (u < T) {
        b = U[(int64_t)u * ms + k];
      } else {
        const int v = task_of(A.coff, T, k);
        b = rr[A.task_off[v] + ((k - A.coff[v]) << cs)];
      }
      acc += a.x * b.x + a.y * b.y;  // Re(conj(a) b)
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0)
      M[t][u] = (u < T ? sqrt(ldexp(1.0, A.m[t] + A.m[u])) : sqrt(ldexp(1.0, A.m[t]))) * acc;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (!A.profile) {
    for (int t = 0; t < T; t++) P->tau_used[t] = P->tau[t];
    return;
  }
  for (int c = 0; c < T; c++) {  // Gaussian elimination with partial pivoting
    int pv = c;
    for (int i = c + 1; i < T; i++)
      if (fabs(M[i][c]) > fabs(M[pv][c])) pv = i;
    for (int k = 0; k <= T; k++) {
      const double tmp = M[c][k];
      M[c][k] = M[pv][k];
      M[pv][k] = tmp;
    }
    for (int i = c + 1; i < T; i++) {
      const double fct = M[i][c] / M[c][c];
      for (int k = c; k <= T; k++) M[i][k] -= fct * M[c][k];
    }
  }
  double tau[MTGP_MAXT];
  for (int c = T - 1; c >= 0; c--) {
    double acc = M[c][T];
    for (int k = c + 1; k < T; k++) acc -= M[c][k] * tau[k];
    tau[c] = acc / M[c][c];
  }
  for (int c = 0; c < T; c++) P->tau_used[c] = tau[c];
}

// partial rows in the solve layout: [q, s, 0 ...]
template <int TM>
__global__ __launch_bounds__(256) void zf_gcv_final_kernel(Alg1Desc A, int64_t N,
                                                           const Params* __restrict__ P,
                                                           const z2* __restrict__ S,
                                                           const z2* __restrict__ rr,
                                                           const z2* __restrict__ U,
                                                           double* __restrict__ partials) {
  constexpr int NQ = 2 + 3 * TM;
  __shared__ double red[4 * NQ];
  double vals[NQ];
#pragma unroll
  for (int q = 0; q < NQ; q++) vals[q] = 0.0;
  for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < N;
       node += (int64_t)gridDim.x * blockDim.x) {
    const int t = task_of(A.task_off, A.T, node);
    const int64_t f = node - A.task_off[t];
    const z2 a = ahat_at(A, P, rr, U, t, f);
    vals[0] += a.x * a.x + a.y * a.y;
    vals[1] += S[pidx(A, t, t, f)].x;
  }
  block_sum_store<NQ>(vals, NQ, red, partials + (size_t)blockIdx.x * NQ);
}

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------
static unsigned grid_for(int64_t items, int64_t cap = 65535) {
  int64_t b = (items + 255) / 256;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

template <int TM>
static void back_stage(bool grad, const Alg1Desc& A1, int t, z2* S, z2* rr, z2* U, double* logs,
                       int* status, hipStream_t st) {
  const dim3 grid(grid_for(1ll << A1.m[t]));
  if (grad)
    hipLaunchKernelGGL((zf_back_kernel<TM, true>), grid, dim3(256), 0, st, A1, t, S, rr, U, logs,
                       status);
  else
    hipLaunchKernelGGL((zf_back_kernel<TM, false>), grid, dim3(256), 0, st, A1, t, S, rr, U, logs,
                       status);
}

template <typename SR>
int launch_zerofill(SR* cols, const Alg1Desc& A1, int64_t N, Params* P, int family, bool grad,
                    const double* yhat, z2* buf, double* logs, double* ahat, double* partials,
                    int* status, hipStream_t st) {
  const int T = A1.T;
  const int64_t ms = A1.msz[T - 1];
  z2* S = buf;
  z2* rr = S + A1.so[T];
  z2* U = rr + N;
  hipLaunchKernelGGL(zf_init_kernel<SR>, dim3(grid_for(A1.so[T] + N + (int64_t)T * ms)), dim3(256),
                     0, st, cols, A1, P, family, N, yhat, S, rr, U);
  const int cs = A1.m[T - 1];
  for (int t = 0; t + 1 < T; t++) {
    for (int u = t + 1; u < T; u++) {
      const int64_t nu = 1ll << A1.m[u];
      const int64_t K = 1ll << (A1.m[t] - A1.m[u]);
      const int G = K >= 64 ? 64 : (int)K;
      const int64_t ntarget = (int64_t)(T - u) * nu + nu + (int64_t)T * (nu >> cs);
      hipLaunchKernelGGL(zf_factor_kernel, dim3(grid_for(ntarget * G)), dim3(256), 0, st, A1, t,
                         u, G, S, rr, U);
    }
  }
  for (int t = T - 1; t >= 0; t--) {
    if (T <= 2) back_stage<2>(grad, A1, t, S, rr, U, logs, status, st);
    else if (T <= 4) back_stage<4>(grad, A1, t, S, rr, U, logs, status, st);
    else if (T <= 8) back_stage<8>(grad, A1, t, S, rr, U, logs, status, st);
    else back_stage<16>(grad, A1, t, S, rr, U, logs, status, st);
  }
  hipLaunchKernelGGL(zf_tau_kernel, dim3(1), dim3(256), 0, st, A1, P, rr, U);
  const dim3 grid((unsigned)zf_final_blocks(N));
#define MTGP_ZFIN(TMV)                                                                          \
  hipLaunchKernelGGL((zf_final_kernel<SR, TMV>), grid, dim3(256), 0, st, cols, A1, N, P, family, \
                     grad ? 1 : 0, yhat, S, rr, U, ahat, partials)
  if (T <= 2) MTGP_ZFIN(2);
  else if (T <= 4) MTGP_ZFIN(4);
  else if (T <= 8) MTGP_ZFIN(8);
  else MTGP_ZFIN(16);
#undef MTGP_ZFIN
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename SR>
int launch_zerofill_gcv(SR* cols, const Alg1Desc& A1, int64_t N, Params* P, int family,
                        const double* yhat, z2* buf, double* logs, double* partials, int* status,
                        hipStream_t st) {
  const int T = A1.T;
  const int64_t ms = A1.msz[T - 1];
  z2* S = buf;
  z2* rr = S + A1.so[T];
  z2* U = rr + N;
  hipLaunchKernelGGL(zf_init_kernel<SR>, dim3(grid_for(A1.so[T] + N + (int64_t)T * ms)), dim3(256),
                     0, st, cols, A1, P, family, N, yhat, S, rr, U);
  const int cs = A1.m[T - 1];
  for (int t = 0; t + 1 < T; t++) {
    for (int u = t + 1; u < T; u++) {
      const int64_t nu = 1ll << A1.m[u];
      const int64_t K = 1ll << (A1.m[t] - A1.m[u]);
      const int G = K >= 64 ? 64 : (int)K;
      const int64_t ntarget = (int64_t)(T - u) * nu + nu + (int64_t)T * (nu >> cs);
      hipLaunchKernelGGL(zf_factor_kernel, dim3(grid_for(ntarget * G)), dim3(256), 0, st, A1, t,
                         u, G, S, rr, U);
    }
  }
  for (int t = T - 1; t >= 0; t--) {
    if (T <= 2) back_stage<2>(true, A1, t, S, rr, U, logs, status, st);
    else if (T <= 4) back_stage<4>(true, A1, t, S, rr, U, logs, status, st);
    else if (T <= 8) back_stage<8>(true, A1, t, S, rr, U, logs, status, st);
    else back_stage<16>(true, A1, t, S, rr, U, logs, status, st);
  }
  hipLaunchKernelGGL(zf_gcv_tau_kernel, dim3(1), dim3(256), 0, st, A1, P, rr, U);
  const dim3 grid((unsigned)zf_final_blocks(N));
  if (T <= 2)
    hipLaunchKernelGGL(zf_gcv_final_kernel<2>, grid, dim3(256), 0, st, A1, N, P, S, rr, U, partials);
  else if (T <= 4)
    hipLaunchKernelGGL(zf_gcv_final_kernel<4>, grid, dim3(256), 0, st, A1, N, P, S, rr, U, partials);
  else if (T <= 8)
    hipLaunchKernelGGL(zf_gcv_final_kernel<8>, grid, dim3(256), 0, st, A1, N, P, S, rr, U, partials);
  else
    hipLaunchKernelGGL(zf_gcv_final_kernel<16>, grid, dim3(256), 0, st, A1, N, P, S, rr, U,
                       partials);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_zerofill_gcv<double>(double*, const Alg1Desc&, int64_t, Params*, int,
                                         const double*, z2*, double*, double*, int*, hipStream_t);
template int launch_zerofill_gcv<float>(float*, const Alg1Desc&, int64_t, Params*, int,
                                        const double*, z2*, double*, double*, int*, hipStream_t);
template int launch_zerofill<double>(double*, const Alg1Desc&, int64_t, Params*, int, bool,
                                     const double*, z2*, double*, double*, double*, int*,
                                     hipStream_t);
template int launch_zerofill<float>(float*, const Alg1Desc&, int64_t, Params*, int, bool,
                                    const double*, z2*, double*, double*, double*, int*,
                                    hipStream_t);

}  // namespace mtgp

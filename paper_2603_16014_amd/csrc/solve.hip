// Per-frequency factorisation for equal sample sizes, parameter decoding and
// the final reductions / chain rule.
//
// Equal sizes (Corollary on equal sample sizes): Lambda is block diagonal
// over frequencies f, each block the T x T matrix
//   Lambda(f)_tu = R_tu lambda_{p(t,u)}(f) + delta_tu xi_t
// with lambda_p the transform of kernel column p.  One thread per frequency
// factors it (Cholesky, FP64), accumulates log det and the quadratic form of
// rhat(f) = yhat(f) - delta_{f0} sqrt(n) tau, and for the gradient forms
// W(f) = Lambda(f)^-1 - ahat ahat^T and the adjoint weights
//   omega_diag(f) = sum_t R_tt W_tt(f),  omega_tu(f) = 2 W_tu(f)  (t < u)
// written over the column buffer (R_tu is applied to the pair column's
// derivative sums in the chain rule), plus G_tt = sum_f W_tt(f) lambda_tt(f)
// (dL/dR_tt) and sum_f W_tt(f) (dL/dxi_t).
// With profiled means and equal sizes, tau_hat_t = yhat_t(0) / sqrt(n), the
// per-task sample mean (Theorem "Fast MTGP computations", item 4 with
// Pi = n Lambda(0)^-1), so rhat(0) = 0.
#include "kernels.h"
#include "solve_dev.h"

namespace mtgp {

__global__ void prep_kernel(const double* __restrict__ theta, Params* __restrict__ P, KDesc kd,
                            int* __restrict__ status) {
  if (blockIdx.x != 0) return;
  prep_device(theta, P, kd, status);
}

__global__ void clear_status_kernel(int* status) {
  if (threadIdx.x == 0) {
    status[0] = 0;
    status[1] = 0;
    *reinterpret_cast<unsigned long long*>(status + 2) = ~0ull;
  }
}

// A fill kernel rather than a memset, so a captured graph holds no memset node.
int launch_clear_status(int* status, hipStream_t st) {
  hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(64), 0, st, status);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prep(const double* theta, Params* P, const KDesc& kd, int* status, hipStream_t st) {
  hipLaunchKernelGGL(prep_kernel, dim3(1), dim3(64), 0, st, theta, P, kd, status);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}


template <int TM>
__device__ constexpr int pk(int i, int j) {
  return i * (i + 1) / 2 + j;
}

// One thread per frequency f (grid solve_blocks(n) x 256).  Lambda(f) = L D L^T
// (unit lower L, FP64): log det = sum log D_j, quad = sum z_j^2 / D_j with
// L z = rhat, ahat = L^-T (z / D), Lambda^-1 = L^-T D^-1 L^-1; eight
// reciprocals and no square roots per frequency.  Per-block sums go to
// partials[block][solve_ns(T)] in the layout of solve_ns, TM = solve_tm(T)
// (T padded to 1/2/4/8/16); ahat_t(0) is nonzero in block 0 only.
// FP32 storage: four waves per SIMD (at most 128 VGPRs, no spill with the
// right-hand side held in FP32).  FP64 storage: three (no spill; four spill
// 28 bytes per lane, which moves 0.9 GB through the caches per 2^24
// frequencies and measured 2% slower).
template <typename Real, int TM, bool GRAD>
__global__ __launch_bounds__(256, sizeof(Real) == 8 ? 3 : 4) void solve_eq_kernel(Real* __restrict__ cols, int64_t n,
                                                       PairMap pm, const Real* __restrict__ yhat,
                                                       const double* __restrict__ yhat0,
                                                       const Params* __restrict__ P, KDesc kd,
                                                       double* __restrict__ partials,
                                                       double* __restrict__ ahat,
                                                       int* __restrict__ status) {
  constexpr int NQ = 2 + 3 * TM, NR = 2 + 2 * TM;  // row size, block-summed slots
  __shared__ double red[4 * NR];
  const int T = kd.T;
  double* row = partials + (size_t)blockIdx.x * NQ;
  // the ahat(0) slots: zero in every row; the frequency-0 thread (thread 0
  // of block 0) overwrites row 0's below
  if (threadIdx.x == 0)
    for (int q = NR; q < NQ; q++) row[q] = 0.0;
  double vals[NR];
#pragma unroll
  for (int q = 0; q < NR; q++) vals[q] = 0.0;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f < n) {
    constexpr int NP = TM * (TM + 1) / 2;
    // every load first and without branches (a load behind a branch of its
    // own is waited for before the next one issues); rows past T read the
    // diagonal column and become identity rows below.  Equal sizes: every
    // diagonal pair uses the one diagonal column.
    const double lam0 = (double)cols[(int64_t)pm.at(0, 0) * n + f];
    Real lv[NP];
    Real yv[TM];
#pragma unroll
    for (int i = 0; i < TM; i++) {
#pragma unroll
      for (int j = 0; j < i; j++) {
        const int ci = i < T ? pm.at(j, i) : pm.at(0, 0);
        lv[pk<TM>(i, j)] = cols[(int64_t)ci * n + f];
      }
      yv[i] = yhat[(int64_t)(i < T ? i : 0) * n + f];
    }
    double A[NP];
#pragma unroll
    for (int i = 0; i < TM; i++) {
      const bool in = i < T;
#pragma unroll
      for (int j = 0; j <= i; j++) {
        const double l = i == j ? lam0 : (double)lv[pk<TM>(i, j)];
        const double a = P->R[j * MTGP_MAXT + i] * l + (i == j ? P->xi[i] : 0.0);
        A[pk<TM>(i, j)] = in ? a : (i == j ? 1.0 : 0.0);
      }
      // right-hand side held at the storage precision until use; frequency 0
      // is formed from the FP64 transform (the means are subtracted from it)
      // and rounded once
      if (f == 0)
        yv[i] = (Real)(kd.profile ? 0.0
                                  : yhat0[(int64_t)(i < T ? i : 0) * n] -
                                        sqrt((double)n) * P->tau[i]);
      if (!in) yv[i] = (Real)0;
    }
    // L D L^T in place: strictly lower part of A becomes L
    double invD[TM], Dv[TM];
    double prod = 1.0;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < TM; j++) {
      double u[TM];
      double dj = A[pk<TM>(j, j)];
#pragma unroll
      for (int k = 0; k < j; k++) {
        u[k] = A[pk<TM>(j, k)] * Dv[k];  // L_jk D_k
        dj -= A[pk<TM>(j, k)] * u[k];
      }
      ok = ok && (dj > 0.0);
      prod *= dj;
      Dv[j] = dj;
      invD[j] = 1.0 / dj;
#pragma unroll
      for (int i = j + 1; i < TM; i++) {
        double v = A[pk<TM>(i, j)];
#pragma unroll
        for (int k = 0; k < j; k++) v -= A[pk<TM>(i, k)] * u[k];
        A[pk<TM>(i, j)] = v * invD[j];
      }
    }
    if (!ok || !isfinite(prod)) flag_bad(status, f);
    vals[1] += log(prod);
    // L z = r; quad = sum z^2 / D; L^T a = z / D
    double a[TM];
    double quad = 0.0;
#pragma unroll
    for (int i = 0; i < TM; i++) {
      double v = (double)yv[i];
#pragma unroll
      for (int k = 0; k < i; k++) v -= A[pk<TM>(i, k)] * a[k];
      a[i] = v;
      quad += v * v * invD[i];
    }
    vals[0] += quad;
#pragma unroll
    for (int i = TM - 1; i >= 0; i--) {
      double v = a[i] * invD[i];
#pragma unroll
      for (int k = i + 1; k < TM; k++) v -= A[pk<TM>(k, i)] * a[k];
      a[i] = v;
    }
    if (f == 0) {
#pragma unroll
      for (int i = 0; i < TM; i++) row[NR + i] = a[i];
    }
    if (ahat) {
#pragma unroll
      for (int i = 0; i < TM; i++)
        if (i < T) ahat[(int64_t)i * n + f] = a[i];
    }
    if (GRAD) {
      // X = L^-1 (unit lower) in place, row by row
#pragma unroll
      for (int i = 1; i < TM; i++) {
#pragma unroll
        for (int j = 0; j < i; j++) {
          double v = A[pk<TM>(i, j)];
#pragma unroll
          for (int k = j + 1; k < i; k++) v += A[pk<TM>(i, k)] * A[pk<TM>(k, j)];
          A[pk<TM>(i, j)] = -v;
        }
      }
      double wdiag = 0.0;
#pragma unroll
      for (int u = 0; u < TM; u++) {
#pragma unroll
        for (int t = 0; t <= u; t++) {
          // (Lambda^-1)_tu = sum_{k >= u} X_kt X_ku / D_k, with X_kk = 1
          double v = (t == u ? 1.0 : A[pk<TM>(u, t)]) * invD[u];
#pragma unroll
          for (int k = u + 1; k < TM; k++) v += A[pk<TM>(k, t)] * A[pk<TM>(k, u)] * invD[k];
          const double w = v - a[t] * a[u];
          if (u < T) {
            if (t == u) {
              vals[2 + TM + t] += w;  // times lam0 into vals[2 + t] at the end
              wdiag += P->R[t * MTGP_MAXT + t] * w;
            } else {
              cols[(int64_t)pm.at(t, u) * n + f] = (Real)(2.0 * w);
            }
          }
        }
      }
      cols[(int64_t)pm.at(0, 0) * n + f] = (Real)wdiag;
#pragma unroll
      for (int t = 0; t < TM; t++)
        if (t < T) vals[2 + t] = vals[2 + TM + t] * lam0;
    }
  }
  block_sum_store<NR>(vals, NR, red, row);
}

template <typename Real>
int launch_solve_eq(Real* cols, int64_t n, const PairMap& pm, int ncol, const Real* yhat,
                    const double* yhat0, const Params* P, const KDesc& kd, bool grad,
                    double* partials, double* ahat, int* status, hipStream_t st) {
  (void)ncol;
  const dim3 grid((unsigned)solve_blocks(n)), block(256);
#define MTGP_SOLVE(TMV)                                                                          \
  do {                                                                                           \
    if (grad)                                                                                    \
      hipLaunchKernelGGL((solve_eq_kernel<Real, TMV, true>), grid, block, 0, st, cols, n, pm,    \
                         yhat, yhat0, P, kd, partials, ahat, status);                            \
    else                                                                                         \
      hipLaunchKernelGGL((solve_eq_kernel<Real, TMV, false>), grid, block, 0, st, cols, n, pm,   \
                         yhat, yhat0, P, kd, partials, ahat, status);                            \
  } while (0)
  if (kd.T <= 1) MTGP_SOLVE(1);
  else if (kd.T <= 2) MTGP_SOLVE(2);
  else if (kd.T <= 4) MTGP_SOLVE(4);
  else if (kd.T <= 8) MTGP_SOLVE(8);
  else MTGP_SOLVE(16);
#undef MTGP_SOLVE
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_solve_eq<double>(double*, int64_t, const PairMap&, int, const double*,
                                     const double*, const Params*, const KDesc&, bool, double*,
                                     double*, int*, hipStream_t);
template int launch_solve_eq<float>(float*, int64_t, const PairMap&, int, const float*,
                                    const double*, const Params*, const KDesc&, bool, double*,
                                    double*, int*, hipStream_t);

// FP64 -> storage-precision copy (the data transform read by the solves)
__global__ void narrow_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}
int launch_narrow(const double* in, float* out, int64_t n, hipStream_t st) {
  if (n <= 0) return 0;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)blocks), dim3(256), 0, st, in, out, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------------------
// Lattices: Lambda(f) is Hermitian, Lambda_tu = R_tu lambda_tu(f) for t < u
// (column of the pair, shift Delta_t - Delta_u), Lambda_ut = conj(Lambda_tu),
// diagonal R_tt Re(lambda_0(f)) + xi_t.  Lambda = L D L^H (complex unit lower
// L, real D).  dL = sum_f sum_tu Re(W_ut dLambda_tu) gives
//   omega_tu = 2 R_tu conj(W_tu) (t < u), omega_diag = sum_t R_tt W_tt,
//   G_tu = sum_f Re(conj(W_tu) lambda_tu), same partial layout as the real case.
// ---------------------------------------------------------------------------
struct zc {
  double x, y;
};
__device__ inline zc zmul(zc a, zc b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline zc zmulc(zc a, zc b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }  // a conj(b)
__device__ inline zc zsub(zc a, zc b) { return {a.x - b.x, a.y - b.y}; }
__device__ inline zc zscale(zc a, double s) { return {a.x * s, a.y * s}; }

template <typename SR, int TM, bool GRAD>
__global__ __launch_bounds__(256) void solve_eq_c_kernel(SR* __restrict__ cols, int64_t n,
                                                         PairMap pm,
                                                         const SR* __restrict__ yhat,
                                                         const double* __restrict__ yhat0,
                                                         const Params* __restrict__ P, KDesc kd,
                                                         double* __restrict__ partials,
                                                         double* __restrict__ ahat,
                                                         int* __restrict__ status) {
  constexpr int NP = TM * (TM + 1) / 2;
  constexpr int NQ = 2 + 3 * TM, NR = 2 + 2 * TM;  // row size, block-summed slots
  __shared__ double red[4 * NR];
  const int T = kd.T;
  double* row = partials + (size_t)blockIdx.x * NQ;
  // the ahat(0) slots: zero in every row; the frequency-0 thread (thread 0
  // of block 0) overwrites row 0's below
  if (threadIdx.x == 0)
    for (int q = NR; q < NQ; q++) row[q] = 0.0;
  double vals[NR];
#pragma unroll
  for (int q = 0; q < NR; q++) vals[q] = 0.0;
  const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f < n) {
    // every load first and without branches (see the real solve); equal
    // sizes: every diagonal pair uses the one diagonal column (real)
    const double lam0 = (double)cols[((size_t)pm.at(0, 0) * n + f) * 2];
    SR lv[NP][2];
    zc yv[TM];
#pragma unroll
    for (int i = 0; i < TM; i++) {
#pragma unroll
      for (int j = 0; j < i; j++) {
        const int ci = i < T ? pm.at(j, i) : pm.at(0, 0);
        const size_t at = ((size_t)ci * n + f) * 2;
        lv[pk<TM>(i, j)][0] = cols[at];
        lv[pk<TM>(i, j)][1] = cols[at + 1];
      }
      const size_t ay = ((size_t)(i < T ? i : 0) * n + f) * 2;
      yv[i] = {(double)yhat[ay], (double)yhat[ay + 1]};
    }
    zc A[NP], r[TM];
#pragma unroll
    for (int i = 0; i < TM; i++) {
      const bool in = i < T;
#pragma unroll
      for (int j = 0; j <= i; j++) {
        const zc l = i == j ? zc{lam0, 0.0}
                            : zc{(double)lv[pk<TM>(i, j)][0], (double)lv[pk<TM>(i, j)][1]};
        // lower entry (i, j), i > j: conj(Lambda_ji) = R_ji conj(lambda_ji)
        const double R = P->R[j * MTGP_MAXT + i];
        const zc a = {R * l.x + (i == j ? P->xi[i] : 0.0), -R * l.y};
        A[pk<TM>(i, j)] = in ? a : zc{i == j ? 1.0 : 0.0, 0.0};
      }
      zc y = yv[i];
      // frequency 0 from the FP64 transform (real): the mean is subtracted from it
      if (f == 0)
        y = kd.profile ? zc{0.0, 0.0}
                       : zc{yhat0[(size_t)(i < T ? i : 0) * n * 2] - sqrt((double)n) * P->tau[i],
                            0.0};
      r[i] = in ? y : zc{0.0, 0.0};
    }
    double invD[TM], Dv[TM];
    double prod = 1.0;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < TM; j++) {
      zc u[TM];
      double dj = A[pk<TM>(j, j)].x;
#pragma unroll
      for (int k = 0; k < j; k++) {
        const zc l = A[pk<TM>(j, k)];
        u[k] = zscale(l, Dv[k]);  // L_jk D_k
        dj -= (l.x * l.x + l.y * l.y) * Dv[k];
      }
      ok = ok && (dj > 0.0);
      prod *= dj;
      Dv[j] = dj;
      invD[j] = 1.0 / dj;
#pragma unroll
      for (int i = j + 1; i < TM; i++) {
        zc v = A[pk<TM>(i, j)];
#pragma unroll
        for (int k = 0; k < j; k++) v = zsub(v, zmulc(A[pk<TM>(i, k)], u[k]));  // L_ik conj(L_jk) D_k
        A[pk<TM>(i, j)] = zscale(v, invD[j]);
      }
    }
    if (!ok || !isfinite(prod)) flag_bad(status, f);
    vals[1] += log(prod);
    zc a[TM];
    double quad = 0.0;
#pragma unroll
    for (int i = 0; i < TM; i++) {
      zc v = r[i];
#pragma unroll
      for (int k = 0; k < i; k++) v = zsub(v, zmul(A[pk<TM>(i, k)], a[k]));
      a[i] = v;
      quad += (v.x * v.x + v.y * v.y) * invD[i];
    }
    vals[0] += quad;
#pragma unroll
    for (int i = TM - 1; i >= 0; i--) {
      zc v = zscale(a[i], invD[i]);
#pragma unroll
      for (int k = i + 1; k < TM; k++) {
        const zc l = A[pk<TM>(k, i)];
        v = zsub(v, zmul({l.x, -l.y}, a[k]));  // conj(L_ki) a_k
      }
      a[i] = v;
    }
    if (f == 0) {
#pragma unroll
      for (int i = 0; i < TM; i++) row[NR + i] = a[i].x;
    }
    if (ahat) {
#pragma unroll
      for (int i = 0; i < TM; i++)
        if (i < T) {
          ahat[((size_t)i * n + f) * 2] = a[i].x;
          ahat[((size_t)i * n + f) * 2 + 1] = a[i].y;
        }
    }
    if (GRAD) {
#pragma unroll
      for (int i = 1; i < TM; i++) {
#pragma unroll
        for (int j = 0; j < i; j++) {
          zc v = A[pk<TM>(i, j)];
#pragma unroll
          for (int k = j + 1; k < i; k++) {
            const zc p2 = zmul(A[pk<TM>(i, k)], A[pk<TM>(k, j)]);
            v = {v.x + p2.x, v.y + p2.y};
          }
          A[pk<TM>(i, j)] = {-v.x, -v.y};
        }
      }
      double wdiag = 0.0;
#pragma unroll
      for (int u = 0; u < TM; u++) {
#pragma unroll
        for (int t = 0; t <= u; t++) {
          // (Lambda^-1)_tu = sum_{k >= u} conj(X_kt) X_ku / D_k
          zc v = (t == u) ? zc{invD[u], 0.0} : zscale({A[pk<TM>(u, t)].x, -A[pk<TM>(u, t)].y}, invD[u]);
#pragma unroll
          for (int k = u + 1; k < TM; k++) {
            const zc xt = A[pk<TM>(k, t)], xu = A[pk<TM>(k, u)];
            const zc p2 = zmulc(xu, xt);  // X_ku conj(X_kt)
            v = {v.x + p2.x * invD[k], v.y + p2.y * invD[k]};
          }
          const zc w = zsub(v, zmulc(a[t], a[u]));  // W_tu = Ainv_tu - a_t conj(a_u)
          if (u < T) {
            if (t == u) {
              vals[2 + t] += w.x * lam0;
              vals[2 + TM + t] += w.x;
              wdiag += P->R[t * MTGP_MAXT + t] * w.x;
            } else {
              const size_t at = ((size_t)pm.at(t, u) * n + f) * 2;
              cols[at] = (SR)(2.0 * w.x);
              cols[at + 1] = (SR)(-2.0 * w.y);
            }
          }
        }
      }
      const size_t at0 = ((size_t)pm.at(0, 0) * n + f) * 2;
      cols[at0] = (SR)wdiag;
      cols[at0 + 1] = (SR)0;
    }
  }
  block_sum_store<NR>(vals, NR, red, row);
}

template <typename SR>
int launch_solve_eq_c(SR* cols, int64_t n, const PairMap& pm, const SR* yhat, const double* yhat0,
                      const Params* P, const KDesc& kd, bool grad, double* partials, double* ahat,
                      int* status, hipStream_t st) {
  const dim3 grid((unsigned)solve_blocks(n)), block(256);
#define MTGP_SOLVEC(TMV)                                                                         \
  do {                                                                                           \
    if (grad)                                                                                    \
      hipLaunchKernelGGL((solve_eq_c_kernel<SR, TMV, true>), grid, block, 0, st, cols, n, pm,    \
                         yhat, yhat0, P, kd, partials, ahat, status);                            \
    else                                                                                         \
      hipLaunchKernelGGL((solve_eq_c_kernel<SR, TMV, false>), grid, block, 0, st, cols, n, pm,   \
                         yhat, yhat0, P, kd, partials, ahat, status);                            \
  } while (0)
  if (kd.T <= 1) MTGP_SOLVEC(1);
  else if (kd.T <= 2) MTGP_SOLVEC(2);
  else if (kd.T <= 4) MTGP_SOLVEC(4);
  else if (kd.T <= 8) MTGP_SOLVEC(8);
  else MTGP_SOLVEC(16);
#undef MTGP_SOLVEC
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_solve_eq_c<double>(double*, int64_t, const PairMap&, const double*,
                                       const double*, const Params*, const KDesc&, bool, double*,
                                       double*, int*, hipStream_t);
template int launch_solve_eq_c<float>(float*, int64_t, const PairMap&, const float*,
                                      const double*, const Params*, const KDesc&, bool, double*,
                                      double*, int*, hipStream_t);

// ---------------------------------------------------------------------------
// finalize: deterministic sums of the block partials and the chain rule
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void finalize_kernel(const double* __restrict__ sp, int nsolve,
                                                       const double* __restrict__ cs,
                                                       const ColInfo* __restrict__ ci, int ncol,
                                                       const double* __restrict__ lp, int nld,
                                                       const double* __restrict__ yhat, int64_t n,
                                                       Params* __restrict__ P, KDesc kd,
                                                       double* __restrict__ out3,
                                                       double* __restrict__ grad,
                                                       double* __restrict__ tau_hat) {
  finalize_device(sp, nsolve, cs, ci, ncol, lp, nld, yhat, n, P, kd, out3, grad, tau_hat);
}

// Per-column sums of the adjoint partial table: block c adds the rows
// [row_off, row_off + row_cnt) of column c (fixed order, deterministic).
__global__ __launch_bounds__(256) void colseg_kernel(const double* __restrict__ in,
                                                     const ColInfo* __restrict__ ci, int nq,
                                                     double* __restrict__ out) {
  __shared__ double red[16];
  const int64_t off = ci[blockIdx.x].row_off, cnt = ci[blockIdx.x].row_cnt;
  for (int q = 0; q < nq; q++) {
    double v = 0.0;
    for (int64_t r = threadIdx.x; r < cnt; r += blockDim.x) v += in[(off + r) * nq + q];
    v = block_sum(v, red);
    if (threadIdx.x == 0) out[(size_t)blockIdx.x * nq + q] = v;
  }
}

int launch_colseg(const double* in, const ColInfo* ci, int ncol, int nq, double* out,
                  hipStream_t st) {
  if (ncol <= 0) return 0;
  hipLaunchKernelGGL(colseg_kernel, dim3(ncol), dim3(256), 0, st, in, ci, nq, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// First stage of the deterministic reduction of a [nrows][ncols] table of
// block partials: block b sums rows b, b + nblk, ... into out[b][ncols].
__global__ __launch_bounds__(256) void colsum_kernel(const double* __restrict__ in, int64_t nrows,
                                                     int ncols, double* __restrict__ out) {
  __shared__ double red[16];
  for (int q = 0; q < ncols; q++) {
    double v = 0.0;
    for (int64_t r = blockIdx.x + (int64_t)gridDim.x * threadIdx.x; r < nrows;
         r += (int64_t)gridDim.x * blockDim.x)
      v += in[r * ncols + q];
    v = block_sum(v, red);
    if (threadIdx.x == 0) out[(size_t)blockIdx.x * ncols + q] = v;
  }
}

int launch_colsum(const double* in, int64_t nrows, int ncols, double* out, int nblk,
                  hipStream_t st) {
  hipLaunchKernelGGL(colsum_kernel, dim3(nblk), dim3(256), 0, st, in, nrows, ncols, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_finalize(const double* solve_partials, int nsolve, const double* col_sums,
                    const ColInfo* ci, int ncol, const double* ld_partials, int nld,
                    const double* yhat0, int64_t n, Params* P, const KDesc& kd, double* out3,
                    double* grad, double* tau_hat, hipStream_t st) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, st, solve_partials, nsolve,
                     col_sums, ci, ncol, ld_partials, nld, yhat0, n, P, kd, out3, grad, tau_hat);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mtgp

// Posterior variance of the multitask GP at arbitrary inputs (Eq.
// MTGP_post_mean_cov, covariance part with (t, x) = (t', x')):
//   var(t, x) = R_tt Q(x, x) - k(t, x)^T Ktilde^-1 k(t, x),
//   k(t, x) = (R_tu Q(x, x_uk))_{u, k}.
// With Ktilde = V Lambda V^dagger (Theorem "Fast MTGP computations") the
// quadratic form is khat^H Lambda^-1 khat with khat = V^dagger k, and the
// task-u block of khat is R_tu times the transform of the cross column
// Q(x, x_uk) over the points of task u, a kernel column of the same kind as
// the pair columns with shift Delta_u XOR x (nets) or Delta_u - x (lattices;
// the SI kernel is even), produced by the column generators and forward
// transforms of the loss path and scaled by n_u^-1/2.
//   Equal sizes: per frequency, Lambda(f) = L D L^H, z = L^-1 khat_t(f),
//     quadratic form sum |z|^2 / D, for each variance task t.
//   Nested sizes: the fill-free task-order factor of the loss (pivots and
//     unnormalised columns left in the pattern storage) is applied to the
//     stacked right-hand sides by forward substitution, stage by stage.
#include <algorithm>

#include "kernels.h"

namespace mtgp {

namespace {

__device__ inline z2 zmul(z2 a, z2 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline z2 zmulc(z2 a, z2 b) { return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y}; }

// pattern entry of row (b, g mod n_b), column (a, g), a <= b (the storage of
// the fill-free elimination)
__device__ inline int64_t vpidx(const Alg1Desc& A, int a, int b, int64_t g) {
  return A.so[a] + ((int64_t)(b - a) << A.m[a]) + g;
}

__device__ inline int vtask_of(const int64_t* off, int T, int64_t i) {
  int t = 0;
  while (t + 1 < T && i >= off[t + 1]) t++;
  return t;
}

}  // namespace

// Cross-column shifts of a batch of test points: out[u][m][j] =
// Delta_uj XOR x_mj (nets) or Delta_uj - x_mj (lattices, mod 2^32).
__global__ void var_shifts_kernel(const uint32_t* __restrict__ xs, int64_t Mb,
                                  const uint32_t* __restrict__ taskshift, int T, int d, int family,
                                  uint32_t* __restrict__ out) {
  const int64_t total = (int64_t)T * Mb * d;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(i % d);
    const int64_t m = (i / d) % Mb;
    const int u = (int)(i / (d * Mb));
    const uint32_t a = taskshift[(size_t)u * d + j], x = xs[(size_t)m * d + j];
    out[i] = family == FAM_DSEQ ? (a ^ x) : (a - x);
  }
}

int launch_var_shifts(const uint32_t* xs, int64_t Mb, const uint32_t* taskshift, int T, int d,
                      int family, uint32_t* out, hipStream_t st) {
  const int64_t total = (int64_t)T * Mb * d;
  const unsigned nb = (unsigned)std::min<int64_t>((total + 255) / 256, 1024);
  hipLaunchKernelGGL(var_shifts_kernel, dim3(nb), dim3(256), 0, st, xs, Mb, taskshift, T, d, family,
                     out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Equal sizes.  Grid (nbx, Mb): block column m is test point m of the
// batch, threads stride over the n spectrum positions q (the same layout for
// every column, so the frequency itself is not needed).  mu holds the cross
// spectra [u][m][n] (complex interleaved for lattices).  Writes
// partials[(m nbx + bx) TM + t] = sum_q |L^-1 khat_t(q)|^2 / D over the
// block, with khat_t(q)_u = R_tu mu_um(q) / sqrt(n).
template <typename SR, int TM, bool CPLX>
__global__ __launch_bounds__(256) void var_eq_kernel(const SR* __restrict__ cols, int64_t n,
                                                     PairMap pm, const double* __restrict__ mu,
                                                     int64_t Mb, const Params* __restrict__ P,
                                                     int T, double* __restrict__ partials) {
  constexpr int NP = TM * (TM + 1) / 2;
  __shared__ double red[4 * TM];
  const int64_t m = blockIdx.y;
  const double rs = 1.0 / sqrt((double)n);
  double acc[TM];
#pragma unroll
  for (int t = 0; t < TM; t++) acc[t] = 0.0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    // Lambda(q), lower triangle: (i, i) = R_ii lambda_diag + xi_i, (i, j), i > j:
    // conj(Lambda_ji) = R_ji conj(lambda_ji); padding rows are the identity
    z2 A[NP];
#pragma unroll
    for (int i = 0; i < TM; i++) {
#pragma unroll
      for (int j = 0; j <= i; j++) {
        z2 a = {i == j ? 1.0 : 0.0, 0.0};
        if (i < T) {
          const int c = i == j ? pm.at(0, 0) : pm.at(j, i);
          const size_t at = (size_t)c * n + q;
          const double lx = CPLX ? (double)cols[2 * at] : (double)cols[at];
          const double ly = CPLX && i != j ? (double)cols[2 * at + 1] : 0.0;
          const double R = P->R[j * MTGP_MAXT + i];
          a = {R * lx + (i == j ? P->xi[i] : 0.0), -R * ly};
        }
        A[i * (i + 1) / 2 + j] = a;
      }
    }
    // L D L^H in place (unit lower L below the diagonal, D on it)
    double Dv[TM];
#pragma unroll
    for (int j = 0; j < TM; j++) {
      double dj = A[j * (j + 1) / 2 + j].x;
#pragma unroll
      for (int k = 0; k < j; k++) {
        const z2 l = A[j * (j + 1) / 2 + k];
        dj -= (l.x * l.x + l.y * l.y) * Dv[k];
      }
      Dv[j] = dj;
      const double inv = 1.0 / dj;
#pragma unroll
      for (int i = j + 1; i < TM; i++) {
        z2 v = A[i * (i + 1) / 2 + j];
#pragma unroll
        for (int k = 0; k < j; k++) {
          const z2 lk = A[j * (j + 1) / 2 + k];
          const z2 p = zmulc(A[i * (i + 1) / 2 + k], {lk.x * Dv[k], lk.y * Dv[k]});
          v.x -= p.x;
          v.y -= p.y;
        }
        A[i * (i + 1) / 2 + j] = {v.x * inv, v.y * inv};
      }
    }
    z2 a[TM];
#pragma unroll
    for (int u = 0; u < TM; u++) {
      a[u] = {0.0, 0.0};
      if (u < T) {
        const size_t at = ((size_t)u * Mb + m) * n + q;
        a[u] = CPLX ? z2{mu[2 * at] * rs, mu[2 * at + 1] * rs} : z2{mu[at] * rs, 0.0};
      }
    }
#pragma unroll
    for (int t = 0; t < TM; t++) {
      if (t >= T) continue;
      z2 z[TM];
      double qf = 0.0;
#pragma unroll
      for (int i = 0; i < TM; i++) {
        const double R = P->R[t * MTGP_MAXT + (i < T ? i : 0)];
        z2 v = {R * a[i].x, R * a[i].y};
#pragma unroll
        for (int k = 0; k < i; k++) {
          const z2 p = zmul(A[i * (i + 1) / 2 + k], z[k]);
          v.x -= p.x;
          v.y -= p.y;
        }
        z[i] = v;
        if (i < T) qf += (v.x * v.x + v.y * v.y) / Dv[i];
      }
      acc[t] += qf;
    }
  }
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int t = 0; t < TM; t++) {
    const double s = wave_sum(acc[t]);
    if ((threadIdx.x & 63) == 0) red[wv * TM + t] = s;
  }
  __syncthreads();
  if (threadIdx.x < TM) {
    double s = 0.0;
    for (int w = 0; w < nw; w++) s += red[w * TM + threadIdx.x];
    partials[((size_t)m * gridDim.x + blockIdx.x) * TM + threadIdx.x] = s;
  }
}

template <typename SR>
int launch_var_eq(const SR* cols, int64_t n, const PairMap& pm, int family, const double* mu,
                  int64_t Mb, const Params* P, int T, double* partials, int nbx, hipStream_t st) {
  const dim3 grid((unsigned)nbx, (unsigned)Mb), block(256);
#define MTGP_VEQ(TMV)                                                                          \
  do {                                                                                         \
    if (family == FAM_LAT)                                                                     \
      hipLaunchKernelGGL((var_eq_kernel<SR, TMV, true>), grid, block, 0, st, cols, n, pm, mu, \
                         Mb, P, T, partials);                                                  \
    else                                                                                       \
      hipLaunchKernelGGL((var_eq_kernel<SR, TMV, false>), grid, block, 0, st, cols, n, pm, mu, \
                         Mb, P, T, partials);                                                  \
  } while (0)
  if (T <= 1) MTGP_VEQ(1);
  else if (T <= 2) MTGP_VEQ(2);
  else if (T <= 4) MTGP_VEQ(4);
  else if (T <= 8) MTGP_VEQ(8);
  else MTGP_VEQ(16);
#undef MTGP_VEQ
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_var_eq<double>(const double*, int64_t, const PairMap&, int, const double*,
                                   int64_t, const Params*, int, double*, int, hipStream_t);
template int launch_var_eq<float>(const float*, int64_t, const PairMap&, int, const double*,
                                  int64_t, const Params*, int, double*, int, hipStream_t);

// Nested sizes, right-hand sides: rhs r = m T + t (test point m, variance
// task t) holds, at node (u, f) (natural frequency f of task u, offset
// task_off[u] + f), R_tu mu_um(f) / sqrt(n_u).  mu_u is [Mb][n_u] at
// mu_off[u] (complex for lattices), in the spectrum layout.
__global__ void var_rhs_kernel(const double* __restrict__ mu, Alg1Desc A, int family, int64_t N,
                               int64_t Mb, const Params* __restrict__ P, z2* __restrict__ Y) {
  const int T = A.T;
  const int64_t total = Mb * T * N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t node = i % N, r = i / N;
    const int t = (int)(r % T);
    const int64_t m = r / T;
    const int u = vtask_of(A.task_off, T, node);
    const int64_t f = node - A.task_off[u];
    // cross spectra of task u: Mb columns of n_u values after Mb * task_off[u]
    const int64_t col = Mb * A.task_off[u] + (m << A.m[u]);
    const int64_t pos = col + spec_pos(family, f, A.m[u]);
    const double s = P->R[t * MTGP_MAXT + u] / sqrt(ldexp(1.0, A.m[u]));
    Y[i] = family == FAM_DSEQ ? z2{s * mu[pos], 0.0} : z2{s * mu[2 * pos], s * mu[2 * pos + 1]};
  }
}

// Forward substitution, stage t (all earlier stages applied): for u > t,
// Y(u, g) -= sum_{f < n_t, f = g mod n_u} S_tu[f] Y(t, f) / S_tt[f], the
// same update the factorisation applies to the data right-hand side.
__global__ void var_fwd_kernel(Alg1Desc A, int t, int64_t N, int64_t nrhs,
                               const z2* __restrict__ S, z2* __restrict__ Y) {
  const int T = A.T;
  // targets: nodes of tasks u > t, for every right-hand side
  const int64_t base = A.task_off[t + 1];
  const int64_t span = N - base;
  const int64_t total = nrhs * span;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / span;
    const int64_t node = base + (i - r * span);
    const int u = vtask_of(A.task_off, T, node);
    const int64_t g = node - A.task_off[u];
    const int64_t K = 1ll << (A.m[t] - A.m[u]);
    z2* Yr = Y + r * N;
    z2 acc = {0.0, 0.0};
    for (int64_t j = 0; j < K; j++) {
      const int64_t f = g + (j << A.m[u]);
      const double d = S[vpidx(A, t, t, f)].x;
      const z2 p = zmul(S[vpidx(A, t, u, f)], Yr[A.task_off[t] + f]);
      acc.x += p.x / d;
      acc.y += p.y / d;
    }
    Yr[node].x -= acc.x;
    Yr[node].y -= acc.y;
  }
}

// sum over nodes of |Y|^2 / D for each right-hand side: grid (nbx, nrhs),
// partials[(r nbx + bx)]
__global__ __launch_bounds__(256) void var_quad_kernel(Alg1Desc A, int64_t N,
                                                       const z2* __restrict__ S,
                                                       const z2* __restrict__ Y,
                                                       double* __restrict__ partials) {
  __shared__ double red[4];
  const int64_t r = blockIdx.y;
  const z2* Yr = Y + r * N;
  double acc = 0.0;
  for (int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; node < N;
       node += (int64_t)gridDim.x * blockDim.x) {
    const int t = vtask_of(A.task_off, A.T, node);
    const int64_t f = node - A.task_off[t];
    const double d = S[vpidx(A, t, t, f)].x;
    const z2 y = Yr[node];
    acc += (y.x * y.x + y.y * y.y) / d;
  }
  const double s = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) v += red[w];
    partials[r * gridDim.x + blockIdx.x] = v;
  }
}

int launch_var_nested(const double* mu, const Alg1Desc& A, int family, int64_t N, int64_t Mb,
                      const Params* P, const z2* S, z2* Y, double* partials, int nbx,
                      hipStream_t st) {
  const int T = A.T;
  const int64_t nrhs = Mb * T;
  const unsigned g1 = (unsigned)std::min<int64_t>((nrhs * N + 255) / 256, 4096);
  hipLaunchKernelGGL(var_rhs_kernel, dim3(g1), dim3(256), 0, st, mu, A, family, N, Mb, P, Y);
  for (int t = 0; t + 1 < T; t++) {
    const int64_t span = N - A.task_off[t + 1];
    const unsigned g = (unsigned)std::min<int64_t>((nrhs * span + 255) / 256, 4096);
    hipLaunchKernelGGL(var_fwd_kernel, dim3(g), dim3(256), 0, st, A, t, N, nrhs, S, Y);
  }
  hipLaunchKernelGGL(var_quad_kernel, dim3((unsigned)nbx, (unsigned)nrhs), dim3(256), 0, st, A, N,
                     S, Y, partials);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// var[m][t] = R_tt Q(x, x) - (sum of the nbx partial quadratic forms of
// (m, t)); partial row of (m, t) at (m rowm + t) nbx, stride 1 over blocks
// (nested) or at (m nbx + bx) rowm + t (equal: stride rowm).  Q(x, x) =
// gamma prod_j (1 + eta_j K(0)) for both kernel families.
__global__ void var_finalize_kernel(const double* __restrict__ partials, int nbx, int64_t Mb,
                                    int rowm, int equal, const Params* __restrict__ P, KDesc kd,
                                    double* __restrict__ var) {
  const int T = kd.T;
  double q0 = P->gamma;
  for (int j = 0; j < kd.d; j++) {
    double k0;
    if (kd.family == FAM_LAT) k0 = univ_value<double, FAM_LAT, 0>(kd.order, 0u, P);
    else if (kd.adaptive) k0 = univ_value<double, FAM_DSEQ, 1>(kd.order, 0u, P);
    else k0 = univ_value<double, FAM_DSEQ, 0>(kd.order, 0u, P);
    q0 *= 1.0 + P->eta[j] * k0;
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < Mb * T;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = i / T;
    const int t = (int)(i - m * T);
    double s = 0.0;
    for (int b = 0; b < nbx; b++)
      s += equal ? partials[((size_t)m * nbx + b) * rowm + t] : partials[(size_t)i * nbx + b];
    var[i] = P->R[t * MTGP_MAXT + t] * q0 - s;
  }
}

int launch_var_finalize(const double* partials, int nbx, int64_t Mb, int rowm, bool equal,
                        const Params* P, const KDesc& kd, double* var, hipStream_t st) {
  const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((Mb * kd.T + 255) / 256, 1024));
  hipLaunchKernelGGL(var_finalize_kernel, dim3(g), dim3(256), 0, st, partials, nbx, Mb, rowm,
                     equal ? 1 : 0, P, kd, var);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mtgp

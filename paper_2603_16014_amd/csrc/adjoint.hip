// Adjoint pass: low-bit Walsh-Hadamard stages of the adjoint weights fused
// with the derivative reduction of the kernel columns.
//
// With Ktilde = V Lambda V^dagger and V independent of theta,
//   dL/dtheta = sum_f trace(W(f) dLambda(f)),  W = Lambda^-1 - ahat ahat^dagger
// (ahat = Lambda^-1 rhat).  Lambda's entries are R_tu times transforms of
// kernel columns c_p, so the column part of the gradient is
//   sum_p sum_i w_p(i) dc_p(i)/dtheta,  w_p = (transform of omega_p)
// where omega_p collects R-weighted W entries of every pair using column p
// (solve kernel).  This kernel finishes the transform of omega_p over the low
// index bits, regenerates c_p's factors in registers and accumulates
//   dc/dlog eta_j = gamma eta_j K_j prod_{k != j} (1 + eta_k K_k)
// with prefix / suffix products (no division: a factor 1 + eta K may be 0),
// plus dc/dlog b_alpha for the adaptive kernel and c itself (dc/dlog gamma).
#include "kernels.h"

namespace mtgp {

template <typename Real, int FAM, int ADAPT, int D>
__global__ __launch_bounds__(256) void adj_reduce_kernel(const Real* __restrict__ base,
                                                         int64_t col_stride, int m, int LB,
                                                         const uint32_t* __restrict__ gen,
                                                         const uint32_t* __restrict__ colshift,
                                                         const Params* __restrict__ P, KDesc kd,
                                                         double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  const int nb = 1 << LB;
  const int E = nb > 256 ? nb / 256 : 1;
  const int d = kd.d;
  uint32_t* S = reinterpret_cast<uint32_t*>(smem);
  Real* lds = reinterpret_cast<Real*>(smem + sizeof(uint32_t) * MAXE * MTGP_MAXD);
  const int col = blockIdx.y;
  const uint32_t i0 = (uint32_t)blockIdx.x << LB;
  const uint32_t t = threadIdx.x;
  const uint32_t* sh = colshift + (size_t)col * d;
  const Real* w = base + (size_t)col * col_stride + i0;
  const int stride = lds_stride(LB);
  for (int i = threadIdx.x; i < nb; i += blockDim.x) lds[lds_at(0, stride, i)] = w[i];
  for (int q = threadIdx.x; q < E * d; q += blockDim.x) {
    const int k = q / d, j = q - k * d;
    const uint32_t idx = i0 + 256u * (uint32_t)k;
    S[k * d + j] = (FAM == FAM_DSEQ) ? (dseq_z(gen + 32 * j, idx) ^ sh[j])
                                     : (lat_z(gen[j], idx, m) + sh[j]);
  }
  lds_fwht<Real>(lds, 1, LB, stride);

  uint32_t a[D];
  Real eta[D];
#pragma unroll
  for (int j = 0; j < D; j++) {
    if (j < d) {
      a[j] = (FAM == FAM_DSEQ) ? dseq_z(gen + 32 * j, t) : lat_z(gen[j], t, m);
      eta[j] = RT<Real>::eta(P, j);
    } else {
      a[j] = 0;
      eta[j] = 0;
    }
  }
  const Real gam = RT<Real>::gamma(P);
  Real acc_eta[D];
  Real acc_b[4] = {0, 0, 0, 0};
  Real acc_c = 0;
#pragma unroll
  for (int j = 0; j < D; j++) acc_eta[j] = 0;

  for (int k = 0; k < E; k++) {
    const int idx = (int)t + 256 * k;
    if (idx >= nb) break;
    const Real wv = lds[lds_at(0, stride, idx)];
    Real K[D], f[D];
    Real Ka[ADAPT ? D : 1][4];
#pragma unroll
    for (int j = 0; j < D; j++) {
      if (j < d) {
        const uint32_t s = S[k * d + j];
        const uint32_t u = (FAM == FAM_DSEQ) ? (a[j] ^ s) : (a[j] + s);
        if (ADAPT) {
          dsi_khat_all<Real>(u, Ka[ADAPT ? j : 0]);
          K[j] = RT<Real>::bw(P, 0) * Ka[ADAPT ? j : 0][0] + RT<Real>::bw(P, 1) * Ka[ADAPT ? j : 0][1] +
                 RT<Real>::bw(P, 2) * Ka[ADAPT ? j : 0][2] + RT<Real>::bw(P, 3) * Ka[ADAPT ? j : 0][3];
        } else {
          K[j] = univ<Real, FAM>(kd.order, u);
        }
        f[j] = (Real)1 + eta[j] * K[j];
      } else {
        K[j] = 0;
        f[j] = 1;
      }
    }
    // prefix products pre[j] = prod_{k<j} f_k, kept in place of a running value
    Real pre[D];
    Real run = gam * wv;
#pragma unroll
    for (int j = 0; j < D; j++) {
      pre[j] = run;
      run *= f[j];
    }
    acc_c += run;  // w * c
    Real suf = 1;
#pragma unroll
    for (int j = D - 1; j >= 0; j--) {
      if (j < d) {
        const Real ps = pre[j] * suf;  // w gamma prod_{k != j} f_k
        acc_eta[j] += ps * eta[j] * K[j];
        if (ADAPT) {
#pragma unroll
          for (int q = 0; q < 4; q++) acc_b[q] += ps * eta[j] * Ka[ADAPT ? j : 0][q];
        }
        suf *= f[j];
      }
    }
  }
  const int nq = adj_nq(d);
  double* out = partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * nq;
  // layout: [0] w c (gamma), [1..d] eta_j, [d+1..d+4] b_alpha (without the b factor)
  double v = block_sum((double)acc_c, red);
  if (threadIdx.x == 0) out[0] = v;
#pragma unroll
  for (int j = 0; j < D; j++) {
    if (j < d) {
      v = block_sum((double)acc_eta[j], red);
      if (threadIdx.x == 0) out[1 + j] = v;
    }
  }
  for (int q = 0; q < 4; q++) {
    v = ADAPT ? block_sum((double)acc_b[q], red) : 0.0;
    if (threadIdx.x == 0) out[1 + d + q] = v;
  }
}

template <typename Real>
int launch_adj_reduce(const Real* base, int64_t col_stride, int ncols, int m, const uint32_t* gen,
                      const uint32_t* colshift, const Params* P, const KDesc& kd, double* partials,
                      const Sched& sc, hipStream_t st) {
  if (ncols <= 0) return 0;
  const int LB = sc.lb(m);
  const size_t lds = gen_cols_lds_bytes(LB, sizeof(Real));
  dim3 grid(1u << (m - LB), (unsigned)ncols);
#define MTGP_ADJ(F, A, DD)                                                                      \
  hipLaunchKernelGGL((adj_reduce_kernel<Real, F, A, DD>), grid, dim3(256), lds, st, base,       \
                     col_stride, m, LB, gen, colshift, P, kd, partials)
#define MTGP_ADJ_D(F, A)                                       \
  do {                                                         \
    if (kd.d <= 4) MTGP_ADJ(F, A, 4);                          \
    else if (kd.d <= 8) MTGP_ADJ(F, A, 8);                     \
    else if (kd.d <= 12) MTGP_ADJ(F, A, 12);                   \
    else if (kd.d <= 16) MTGP_ADJ(F, A, 16);                   \
    else MTGP_ADJ(F, A, 32);                                   \
  } while (0)
  if (kd.family == FAM_DSEQ) {
    if (kd.adaptive) MTGP_ADJ_D(FAM_DSEQ, 1); else MTGP_ADJ_D(FAM_DSEQ, 0);
  } else {
    MTGP_ADJ_D(FAM_LAT, 0);
  }
#undef MTGP_ADJ_D
#undef MTGP_ADJ
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_adj_reduce<double>(const double*, int64_t, int, int, const uint32_t*,
                                       const uint32_t*, const Params*, const KDesc&, double*,
                                       const Sched&, hipStream_t);
template int launch_adj_reduce<float>(const float*, int64_t, int, int, const uint32_t*,
                                      const uint32_t*, const Params*, const KDesc&, double*,
                                      const Sched&, hipStream_t);

}  // namespace mtgp

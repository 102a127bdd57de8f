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
#include "colgen.h"

namespace mtgp {

template <typename Real, typename TIn, int KT, int D>
__global__ __launch_bounds__(256) void adj_reduce_kernel(const TIn* __restrict__ base,
                                                         int64_t col_stride, int m, int LB,
                                                         const uint32_t* __restrict__ gen,
                                                         const uint32_t* __restrict__ colshift,
                                                         const Params* __restrict__ P, int d,
                                                         double* __restrict__ partials) {
  constexpr int FAM = kt_family(KT);
  constexpr bool ADAPT = KT == KT_DSIA;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  Real* lds = reinterpret_cast<Real*>(smem);
  const int nb = 1 << LB;
  const int E = nb > 256 ? nb >> 8 : 1;
  const int col = blockIdx.y;
  const uint32_t i0 = (uint32_t)blockIdx.x << LB;
  const uint32_t t = threadIdx.x;
  const TIn* w = base + (size_t)col * col_stride + i0;
  const int stride = lds_stride(LB);
  for (int i = threadIdx.x; i < nb; i += blockDim.x) lds[lds_at(0, stride, i)] = (Real)w[i];
  lds_fwht<Real>(lds, 1, LB, stride);

  Real acc_eta[D];
  Real acc_b[4] = {0, 0, 0, 0};
  Real acc_c = 0;
#pragma unroll
  for (int j = 0; j < D; j++) acc_eta[j] = 0;
  if ((int)t < nb) {
    Digits<FAM, D> dg;
    dg.init(gen, colshift + (size_t)col * d, d, t, i0, m);
    Real eta[D];
#pragma unroll
    for (int j = 0; j < D; j++) eta[j] = j < d ? RT<Real>::eta(P, j) : (Real)0;
    const Real gam = RT<Real>::gamma(P);
    for (int k = 0; k < E; k++) {
      const Real wv = lds[lds_at(0, stride, (int)t + 256 * dg.elem(k))];
      Real K[D], f[D];
      Real Ka[ADAPT ? D : 1][4];
#pragma unroll
      for (int j = 0; j < D; j++) {
        if (j < d) {
          if constexpr (ADAPT) {
            dsi_khat_all<Real>(dg.u(j), Ka[j]);
            K[j] = RT<Real>::bw(P, 0) * Ka[j][0] + RT<Real>::bw(P, 1) * Ka[j][1] +
                   RT<Real>::bw(P, 2) * Ka[j][2] + RT<Real>::bw(P, 3) * Ka[j][3];
          } else {
            K[j] = kval<Real, KT>(dg.u(j), P);
          }
          f[j] = fma(eta[j], K[j], (Real)1);
        } else {
          K[j] = 0;
          f[j] = 1;
        }
      }
      // pre[j] = w gamma prod_{k<j} f_k; the suffix product runs backwards
      Real pre[D];
      Real run = gam * wv;
#pragma unroll
      for (int j = 0; j < D; j++) {
        pre[j] = run;
        if (j < d) run *= f[j];
      }
      acc_c += run;  // w * c
      Real suf = 1;
#pragma unroll
      for (int j = D - 1; j >= 0; j--) {
        if (j < d) {
          const Real ps = pre[j] * suf * eta[j];  // w gamma eta_j prod_{k != j} f_k
          acc_eta[j] = fma(ps, K[j], acc_eta[j]);
          if constexpr (ADAPT) {
#pragma unroll
            for (int q = 0; q < 4; q++) acc_b[q] = fma(ps, Ka[j][q], acc_b[q]);
          }
          suf *= f[j];
        }
      }
      if (k + 1 < E) dg.advance(gen, d, k);
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

template <typename Real, typename TIn>
int launch_adj_reduce(const TIn* base, int64_t col_stride, int ncols, int m, const uint32_t* gen,
                      const uint32_t* colshift, const Params* P, const KDesc& kd, double* partials,
                      const Sched& sc, hipStream_t st) {
  if (ncols <= 0) return 0;
  const int LB = sc.lb(m);
  const size_t lds = gen_cols_lds_bytes(LB, sizeof(Real));
  const dim3 grid(1u << (m - LB), (unsigned)ncols);
  const int kt = kt_of(kd.family, kd.order, kd.adaptive);
#define MTGP_ADJ(DD, KTV)                                                                         \
  hipLaunchKernelGGL((adj_reduce_kernel<Real, TIn, KTV, DD>), grid, dim3(256), lds, st, base,     \
                     col_stride, m, LB, gen, colshift, P, kd.d, partials)
  switch (kt) {
    case KT_DSI1: MTGP_DISPATCH_D(kd.d, MTGP_ADJ, KT_DSI1); break;
    case KT_DSI2: MTGP_DISPATCH_D(kd.d, MTGP_ADJ, KT_DSI2); break;
    case KT_DSI3: MTGP_DISPATCH_D(kd.d, MTGP_ADJ, KT_DSI3); break;
    case KT_DSI4: MTGP_DISPATCH_D(kd.d, MTGP_ADJ, KT_DSI4); break;
    case KT_DSIA: MTGP_DISPATCH_D(kd.d, MTGP_ADJ, KT_DSIA); break;
    default: return -1;
  }
#undef MTGP_ADJ
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_adj_reduce<double, double>(const double*, int64_t, int, int, const uint32_t*,
                                               const uint32_t*, const Params*, const KDesc&,
                                               double*, const Sched&, hipStream_t);
template int launch_adj_reduce<double, float>(const float*, int64_t, int, int, const uint32_t*,
                                              const uint32_t*, const Params*, const KDesc&,
                                              double*, const Sched&, hipStream_t);
template int launch_adj_reduce<float, float>(const float*, int64_t, int, int, const uint32_t*,
                                             const uint32_t*, const Params*, const KDesc&,
                                             double*, const Sched&, hipStream_t);

}  // namespace mtgp

// Design points and the direct-sum posterior mean.
//
// Points (bit-exact):
//   digital sequence: x_i = (XOR_{p: i_p = 1} g_p) XOR Delta   (Def. "Base-2
//     digitally-shifted digital sequences", radical-inverse order)
//   rank-1 lattice:   x_i = (v(i) g + Delta) mod 1, v(i) = bitrev32(i) 2^-32
//     (Def. "Shifted rank-1 lattice"), so the digit is bitrev32(i) g + Delta
//     modulo 2^32.
// Posterior mean (Eq. MTGP_post_mean_cov):
//   mu(t, x*) = tau_t + sum_u R_tu sum_k Q(x*, x_uk) alpha_uk,
// summed directly over training points regenerated on the fly and staged in
// LDS 256 at a time.  The training points are split into chunks (grid y) so
// that a few thousand test points still fill the GPU; per-chunk partial sums
// are added in a fixed order afterwards.  alpha is given per task in the
// order of the transform
// (radical-inverse order for digital sequences, natural lattice order j with
// point j g / n + Delta for lattices).
#include "colgen.h"

namespace mtgp {

__global__ void gen_points_kernel(const uint32_t* __restrict__ gen,
                                  const uint32_t* __restrict__ shift, int family, int d,
                                  int64_t first, int64_t count, uint32_t* __restrict__ out) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < count;
       q += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t i = (uint32_t)(first + q);
    for (int j = 0; j < d; j++) {
      uint32_t x;
      if (family == FAM_DSEQ) x = dseq_z(gen + 32 * j, i) ^ shift[j];
      else x = __brev(i) * gen[j] + shift[j];
      out[q * d + j] = x;
    }
  }
}

int launch_gen_points(const uint32_t* gen, const uint32_t* shift, int family, int d, int m,
                      int64_t first, int64_t count, uint32_t* out, hipStream_t st) {
  (void)m;
  if (count <= 0) return 0;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  hipLaunchKernelGGL(gen_points_kernel, dim3((unsigned)blocks), dim3(256), 0, st, gen, shift,
                     family, d, first, count, out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// The kernel type and the dimension width are compile-time: each factor is
// f_j = 1 + sc_j kappa_j (the scaled form of the fused column kernels, with
// the order-2 FP64 table in LDS), padding dimensions have sc = 0 and give
// f = 1 exactly.
template <typename Real, int KT, int D>
__global__ __launch_bounds__(256) void predict_direct_kernel(
    const uint32_t* __restrict__ gen, const uint32_t* __restrict__ shifts, PredTasks pt,
    PredChunks pc, const double* __restrict__ alpha, const uint32_t* __restrict__ xs, int64_t M,
    const Params* __restrict__ P, KDesc kd, double* __restrict__ part) {
  constexpr int FAM = kt_family(KT);
  __shared__ uint32_t xk[256 * D];
  __shared__ double ak[256];
  __shared__ Kap2Entry k2tab[uses_kap2_table<Real, KT>() ? 33 : 1];
  if constexpr (uses_kap2_table<Real, KT>()) fill_kap2_table(k2tab);  // ordered by the loop's barriers
  const int d = kd.d;
  const int64_t mi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool active = mi < M;
  // chunk blockIdx.y: task u, training indices [k_lo, k_hi)
  const int c = blockIdx.y;
  int u = 0;
  while (u + 1 < kd.T && pc.cstart[u + 1] <= c) u++;
  const int64_t nu = (int64_t)1 << pt.m[u];
  const int64_t k_lo = (int64_t)(c - pc.cstart[u]) * pc.chunk;
  const int64_t k_hi = k_lo + pc.chunk < nu ? k_lo + pc.chunk : nu;
  uint32_t xm[D];
  Real sc[D];
#pragma unroll
  for (int j = 0; j < D; j++) {
    xm[j] = (active && j < d) ? xs[mi * d + j] : 0u;
    sc[j] = kscale<Real, KT>(j < d ? RT<Real>::eta(P, j) : (Real)0);
  }
  const Real gam = RT<Real>::gamma(P);
  const uint32_t* sh = shifts + (size_t)u * d;
  double acc = 0.0;
  for (int64_t k0 = k_lo; k0 < k_hi; k0 += 256) {
    __syncthreads();
    const int64_t k = k0 + threadIdx.x;
    if (k < k_hi) {
      for (int j = 0; j < D; j++) {
        uint32_t x = 0u;
        if (j < d)
          x = (FAM == FAM_DSEQ) ? (dseq_z(gen + 32 * j, (uint32_t)k) ^ sh[j])
                                : (lat_z(gen[j], (uint32_t)k, pt.m[u]) + sh[j]);
        xk[threadIdx.x * D + j] = x;
      }
      ak[threadIdx.x] = alpha[pt.off[u] + k];
    }
    __syncthreads();
    const int cnt = (k_hi - k0) < 256 ? (int)(k_hi - k0) : 256;
    for (int q = 0; q < cnt; q++) {
      Real qv = gam;
#pragma unroll
      for (int j = 0; j < D; j++) {
        const uint32_t x2 = xk[q * D + j];
        const uint32_t uu = (FAM == FAM_DSEQ) ? (xm[j] ^ x2) : (xm[j] - x2);
        qv *= fma(sc[j], kappa_t<Real, KT>(uu, P, k2tab), (Real)1);
      }
      acc += (double)qv * ak[q];
    }
  }
  if (active) part[(size_t)c * M + mi] = acc;
}

// mean[i][t] = tau_t + sum_c R_{t, u(c)} part[c][i], chunks in a fixed order
__global__ __launch_bounds__(256) void predict_reduce_kernel(const double* __restrict__ part,
                                                             PredChunks pc, int64_t M,
                                                             const Params* __restrict__ P,
                                                             KDesc kd, double* __restrict__ mean) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= M) return;
  const int T = kd.T;
  double su[MTGP_MAXT];
  for (int u = 0; u < T; u++) {
    double s = 0.0;
    for (int c = pc.cstart[u]; c < pc.cstart[u + 1]; c++) s += part[(size_t)c * M + i];
    su[u] = s;
  }
  for (int t = 0; t < T; t++) {
    double v = 0.0;
    for (int u = 0; u < T; u++) v += P->R[t * MTGP_MAXT + u] * su[u];
    mean[i * T + t] = P->tau_used[t] + v;
  }
}

template <typename Real>
int launch_predict_direct(const uint32_t* gen, const uint32_t* shifts, const PredTasks& pt,
                          const PredChunks& pc, const double* alpha, const uint32_t* xs,
                          int64_t M, const Params* P, const KDesc& kd, double* part, double* mean,
                          hipStream_t st) {
  if (M <= 0) return 0;
  const dim3 grid((unsigned)((M + 255) / 256), (unsigned)pc.cstart[kd.T]), block(256);
#define MTGP_PRED(DD, KTV)                                                                       \
  hipLaunchKernelGGL((predict_direct_kernel<Real, KTV, DD>), grid, block, 0, st, gen, shifts,     \
                     pt, pc, alpha, xs, M, P, kd, part)
  switch (kt_of(kd.family, kd.order, kd.adaptive)) {
    case KT_DSI1: MTGP_DISPATCH_D(kd.d, MTGP_PRED, KT_DSI1); break;
    case KT_DSI2: MTGP_DISPATCH_D(kd.d, MTGP_PRED, KT_DSI2); break;
    case KT_DSI3: MTGP_DISPATCH_D(kd.d, MTGP_PRED, KT_DSI3); break;
    case KT_DSI4: MTGP_DISPATCH_D(kd.d, MTGP_PRED, KT_DSI4); break;
    case KT_DSIA: MTGP_DISPATCH_D(kd.d, MTGP_PRED, KT_DSIA); break;
    case KT_SI1: MTGP_DISPATCH_D(kd.d, MTGP_PRED, KT_SI1); break;
    case KT_SI2: MTGP_DISPATCH_D(kd.d, MTGP_PRED, KT_SI2); break;
    case KT_SI3: MTGP_DISPATCH_D(kd.d, MTGP_PRED, KT_SI3); break;
    default: return -1;
  }
#undef MTGP_PRED
  if (hipGetLastError() != hipSuccess) return -1;
  hipLaunchKernelGGL(predict_reduce_kernel, dim3((unsigned)((M + 255) / 256)), block, 0, st, part,
                     pc, M, P, kd, mean);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_predict_direct<double>(const uint32_t*, const uint32_t*, const PredTasks&,
                                           const PredChunks&, const double*, const uint32_t*,
                                           int64_t, const Params*, const KDesc&, double*, double*,
                                           hipStream_t);
template int launch_predict_direct<float>(const uint32_t*, const uint32_t*, const PredTasks&,
                                          const PredChunks&, const double*, const uint32_t*,
                                          int64_t, const Params*, const KDesc&, double*, double*,
                                          hipStream_t);

}  // namespace mtgp

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
#include "kernels.h"

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

template <typename Real, int FAM, int ADAPT, int D>
__global__ __launch_bounds__(256) void predict_direct_kernel(
    const uint32_t* __restrict__ gen, const uint32_t* __restrict__ shifts, PredTasks pt,
    PredChunks pc, const double* __restrict__ alpha, const uint32_t* __restrict__ xs, int64_t M,
    const Params* __restrict__ P, KDesc kd, double* __restrict__ part) {
  __shared__ uint32_t xk[256 * D];
  __shared__ double ak[256];
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
  Real eta[D];
#pragma unroll
  for (int j = 0; j < D; j++) {
    xm[j] = (active && j < d) ? xs[mi * d + j] : 0u;
    eta[j] = j < d ? RT<Real>::eta(P, j) : (Real)0;
  }
  const Real gam = RT<Real>::gamma(P);
  const uint32_t* sh = shifts + (size_t)u * d;
  double acc = 0.0;
  for (int64_t k0 = k_lo; k0 < k_hi; k0 += 256) {
    __syncthreads();
    const int64_t k = k0 + threadIdx.x;
    if (k < k_hi) {
      for (int j = 0; j < d; j++) {
        xk[threadIdx.x * D + j] = (FAM == FAM_DSEQ) ? (dseq_z(gen + 32 * j, (uint32_t)k) ^ sh[j])
                                                    : (lat_z(gen[j], (uint32_t)k, pt.m[u]) + sh[j]);
      }
      ak[threadIdx.x] = alpha[pt.off[u] + k];
    }
    __syncthreads();
    const int cnt = (k_hi - k0) < 256 ? (int)(k_hi - k0) : 256;
    for (int q = 0; q < cnt; q++) {
      Real qv = gam;
#pragma unroll
      for (int j = 0; j < D; j++) {
        // padding slots: eta = 0, so the factor is exactly 1
        const uint32_t x2 = xk[q * D + (j < d ? j : 0)];
        const uint32_t uu = (FAM == FAM_DSEQ) ? (xm[j] ^ x2) : (xm[j] - x2);
        qv = fma(qv * eta[j], univ_value<Real, FAM, ADAPT>(kd.order, uu, P), qv);
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
#define MTGP_PRED(F, A, DD)                                                                      \
  hipLaunchKernelGGL((predict_direct_kernel<Real, F, A, DD>), grid, block, 0, st, gen, shifts,   \
                     pt, pc, alpha, xs, M, P, kd, part)
#define MTGP_PRED_D(F, A)                     \
  do {                                        \
    if (kd.d <= 4) MTGP_PRED(F, A, 4);        \
    else if (kd.d <= 8) MTGP_PRED(F, A, 8);   \
    else if (kd.d <= 12) MTGP_PRED(F, A, 12); \
    else if (kd.d <= 16) MTGP_PRED(F, A, 16); \
    else MTGP_PRED(F, A, 32);                 \
  } while (0)
  if (kd.family == FAM_DSEQ) {
    if (kd.adaptive) MTGP_PRED_D(FAM_DSEQ, 1); else MTGP_PRED_D(FAM_DSEQ, 0);
  } else {
    MTGP_PRED_D(FAM_LAT, 0);
  }
#undef MTGP_PRED_D
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

// Posterior mean on a structured test net.
//
// Digital sequences.  Test points x*_i = z_i XOR Delta*, i < n* = 2^m*, share the generating
// matrices, so each (test net, task u) cross block has the structure of
// Theorem "Fast MTGP computations" with pair shift Delta* XOR Delta_u:
//   K_{*u} alpha_u = V_{m*} v_u with, for f < n*,
//     n* >= n_u (tall): v_u(f) = sqrt(n_u / n*) lambda_u(f) ahat_u(f mod n_u),
//     n* <  n_u (wide): v_u(f) = sqrt(n* / n_u) sum_{g = f mod n*} lambda_u(g) ahat_u(g),
//   where lambda_u is the Walsh-Hadamard transform of the column
//   c_u(i) = Q(z_i XOR Delta* XOR Delta_u), i < max(n*, n_u), and ahat_u =
//   V^dagger alpha_u (the per-frequency solve's output).  Then
//   mu*_t = tau_t + V_{m*} sum_u R_tu v_u  (Eq. MTGP_post_mean_cov), and V_{m*}
//   is the Walsh-Hadamard transform divided by sqrt(n*).
#include "kernels.h"

namespace mtgp {

struct ShiftTable {
  uint32_t s[MTGP_MAXT * MTGP_MAXD];
};

__global__ void prednet_shifts_kernel(ShiftTable tab, int count, uint32_t* __restrict__ out) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) out[i] = tab.s[i];
}

// one thread per test frequency f: w[t][f] = sum_u R_tu v_u(f)
__global__ __launch_bounds__(256) void prednet_fold_kernel(const double* __restrict__ lam,
                                                           PredNet pn, const double* __restrict__ ahat,
                                                           const Params* __restrict__ P,
                                                           double* __restrict__ w) {
  const int64_t ns = (int64_t)1 << pn.m_star;
  const int T = pn.T;
  for (int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f < ns;
       f += (int64_t)gridDim.x * blockDim.x) {
    double v[MTGP_MAXT];
#pragma unroll
    for (int u = 0; u < MTGP_MAXT; u++) {
      v[u] = 0.0;
      if (u < T) {
        const double* lu = lam + pn.col_off[u];
        const double* au = ahat + pn.task_off[u];
        const int mu = pn.m[u];
        if (pn.m_star >= mu) {
          v[u] = sqrt(ldexp(1.0, mu - pn.m_star)) * lu[f] * au[f & (((int64_t)1 << mu) - 1)];
        } else {
          double acc = 0.0;
          for (int64_t g = f; g < ((int64_t)1 << mu); g += ns) acc += lu[g] * au[g];
          v[u] = sqrt(ldexp(1.0, pn.m_star - mu)) * acc;
        }
      }
    }
    for (int t = 0; t < T; t++) {
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < MTGP_MAXT; u++)
        if (u < T) acc += P->R[t * MTGP_MAXT + u] * v[u];
      w[(size_t)t * ns + f] = acc;
    }
  }
}

__global__ void prednet_out_kernel(const double* __restrict__ w, PredNet pn,
                                   const Params* __restrict__ P, double* __restrict__ mean) {
  const int64_t ns = (int64_t)1 << pn.m_star;
  const double s = 1.0 / sqrt((double)ns);
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < ns * pn.T;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q / pn.T;
    const int t = (int)(q - i * pn.T);
    mean[q] = P->tau_used[t] + w[(size_t)t * ns + i] * s;
  }
}

// ---------------------------------------------------------------------------
// Lattices (shift-invariant kernels).  With L_u = max(m*, m_u) both the test
// lattice x*_j = j g / n* + Delta* and task u's lattice x_uj = j g / n_u +
// Delta_u (natural order j) lie in the lattice of 2^L_u points, and the cross
// product is a cyclic convolution there:
//   sum_j Q(x*_j* - x_uj) alpha_u(j) = (c_u (*) alpha_u upsampled)(j* 2^(L_u - m*)),
//   c_u(i) = Q(i g / 2^L_u + Delta* - Delta_u).
// With F the unnormalised DFT of length 2^L_u, the upsampled alpha_u has
// spectrum sqrt(n_u) ahat_u(f mod n_u) (ahat_u = n_u^-1/2 F alpha_u), and the
// samples at the test lattice fold the frequencies mod n*:
//   v_u(f') = 2^-L_u sum_{f = f' mod n*} C_u(f) sqrt(n_u) ahat_u(f mod n_u),
//   mu*_t(x*_j*) = tau_t + Re sum_{f' < n*} e^{2 pi i f' j* / n*} sum_u R_tu v_u(f')
// (Eq. MTGP_post_mean_cov).  Spectra sit at bit-reversed positions; the last
// sum is the lattice adjoint transform of conj(w), in natural order j*.
// ---------------------------------------------------------------------------
__device__ inline int64_t brev_pos(int64_t f, int m) {
  return m ? (int64_t)(__brevll((unsigned long long)f) >> (64 - m)) : 0;
}

// one thread per test frequency f': w[t] at position bitrev_m*(f') (complex)
__global__ __launch_bounds__(256) void prednet_lat_fold_kernel(const double* __restrict__ lam,
                                                               PredNet pn,
                                                               const double* __restrict__ ahat,
                                                               const Params* __restrict__ P,
                                                               double* __restrict__ w) {
  const int64_t ns = (int64_t)1 << pn.m_star;
  const int T = pn.T;
  for (int64_t f0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; f0 < ns;
       f0 += (int64_t)gridDim.x * blockDim.x) {
    double vr[MTGP_MAXT], vi[MTGP_MAXT];
#pragma unroll
    for (int u = 0; u < MTGP_MAXT; u++) {
      vr[u] = 0.0;
      vi[u] = 0.0;
      if (u < T) {
        const int mu = pn.m[u];
        const int L = pn.m_star > mu ? pn.m_star : mu;
        const double* lu = lam + pn.col_off[u];
        double ar = 0.0, ai = 0.0;
        for (int64_t f = f0; f < ((int64_t)1 << L); f += ns) {
          const int64_t pc = brev_pos(f, L);
          const int64_t pa = pn.task_off[u] + brev_pos(f & (((int64_t)1 << mu) - 1), mu);
          const double cr = lu[2 * pc], ci = lu[2 * pc + 1];
          const double yr = ahat[2 * pa], yi = ahat[2 * pa + 1];
          ar += cr * yr - ci * yi;
          ai += cr * yi + ci * yr;
        }
        const double sc = sqrt(ldexp(1.0, mu)) * ldexp(1.0, -L);
        vr[u] = ar * sc;
        vi[u] = ai * sc;
      }
    }
    const int64_t pos = brev_pos(f0, pn.m_star);
    for (int t = 0; t < T; t++) {
      double accr = 0.0, acci = 0.0;
#pragma unroll
      for (int u = 0; u < MTGP_MAXT; u++)
        if (u < T) {
          accr += P->R[t * MTGP_MAXT + u] * vr[u];
          acci += P->R[t * MTGP_MAXT + u] * vi[u];
        }
      w[2 * ((size_t)t * ns + pos)] = accr;
      w[2 * ((size_t)t * ns + pos) + 1] = acci;
    }
  }
}

// mean[i][t] = tau_t + u_t(bitrev_m*(i)): test point i in radical-inverse order
__global__ void prednet_lat_out_kernel(const double* __restrict__ ureal, PredNet pn,
                                       const Params* __restrict__ P, double* __restrict__ mean) {
  const int64_t ns = (int64_t)1 << pn.m_star;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < ns * pn.T;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q / pn.T;
    const int t = (int)(q - i * pn.T);
    mean[q] = P->tau_used[t] + ureal[(size_t)t * ns + brev_pos(i, pn.m_star)];
  }
}

int launch_prednet_lat_fold(const double* lam, const PredNet& pn, const double* ahat,
                            const Params* P, double* w, hipStream_t st) {
  const int64_t ns = (int64_t)1 << pn.m_star;
  int64_t blocks = (ns + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(prednet_lat_fold_kernel, dim3((unsigned)blocks), dim3(256), 0, st, lam, pn,
                     ahat, P, w);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prednet_lat_out(const double* ureal, const PredNet& pn, const Params* P, double* mean,
                           hipStream_t st) {
  const int64_t total = ((int64_t)1 << pn.m_star) * pn.T;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(prednet_lat_out_kernel, dim3((unsigned)blocks), dim3(256), 0, st, ureal, pn,
                     P, mean);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prednet_shifts(const uint32_t* host_shifts, int count, uint32_t* dev,
                          hipStream_t st) {
  ShiftTable tab;
  for (int i = 0; i < count; i++) tab.s[i] = host_shifts[i];
  hipLaunchKernelGGL(prednet_shifts_kernel, dim3(1), dim3(256), 0, st, tab, count, dev);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prednet_fold(const double* lam, const PredNet& pn, const double* ahat, const Params* P,
                        double* w, hipStream_t st) {
  const int64_t ns = (int64_t)1 << pn.m_star;
  int64_t blocks = (ns + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(prednet_fold_kernel, dim3((unsigned)blocks), dim3(256), 0, st, lam, pn, ahat,
                     P, w);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prednet_out(const double* w, const PredNet& pn, const Params* P, double* mean,
                       hipStream_t st) {
  const int64_t total = ((int64_t)1 << pn.m_star) * pn.T;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(prednet_out_kernel, dim3((unsigned)blocks), dim3(256), 0, st, w, pn, P, mean);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mtgp

// On-device Adam update of the packed hyperparameter vector (the optimiser
// that drives loss + gradient evaluations; the paper fits by a first-order
// method on the same loss).  The step counter lives in device memory so the
// update can be replayed inside a captured HIP graph.
#include "kernels.h"

namespace mtgp {

__global__ void adam_kernel(double* __restrict__ theta, const double* __restrict__ grad,
                            double* __restrict__ m1, double* __restrict__ m2, int64_t n, double lr,
                            double b1, double b2, double eps, int64_t* __restrict__ step,
                            const uint8_t* __restrict__ frozen) {
  const int64_t k = *step + 1;
  const double c1 = 1.0 - pow(b1, (double)k), c2 = 1.0 - pow(b2, (double)k);
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    if (frozen && frozen[i]) continue;
    const double g = grad[i];
    const double a = b1 * m1[i] + (1.0 - b1) * g;
    const double b = b2 * m2[i] + (1.0 - b2) * g * g;
    m1[i] = a;
    m2[i] = b;
    theta[i] -= lr * (a / c1) / (sqrt(b / c2) + eps);
  }
  __syncthreads();
  if (threadIdx.x == 0) *step = k;
}

int launch_adam(double* theta, const double* grad, double* m1, double* m2, int64_t n, double lr,
                double b1, double b2, double eps, int64_t* step, const uint8_t* frozen,
                hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3(1), dim3(256), 0, st, theta, grad, m1, m2, n, lr, b1, b2,
                     eps, step, frozen);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mtgp

// Lattice kernel columns and their derivative sums at natural lattice index
// j (point j g / n + shift): the column value, the eta K factor of the
// shift-invariant Bernoulli kernels, and the per-thread derivative
// accumulator of the adjoint reduction.  Shared by the lattice transform
// passes (lattice.hip) and the many-fit kernels (batch.hip).
#pragma once
#include "colgen.h"

namespace mtgp {

// lattice kernel column value at natural index j of a column with shift sh
template <typename R, int KT>
__device__ inline R lat_col_value(const uint32_t* __restrict__ gen, const uint32_t* __restrict__ sh,
                                  int d, uint32_t j, int m, const Params* __restrict__ P) {
  R c = RT<R>::gamma(P);
  for (int q = 0; q < d; q++)
    c = fma(c * RT<R>::eta(P, q), kval<R, KT>(lat_z(gen[q], j, m) + sh[q], P), c);
  return c;
}

// eta K of the shift-invariant kernels in y = x (x - 1), x = u 2^-32:
//   order 1: B2 = y + 1/6,   order 2: B4 = y^2 - 1/30,
//   order 3: B6 = y^2 (y - 1/2) + 1/42,
// so that eta K = fma(ka, p(y), kb) with per-dimension constants
// ka = eta c_alpha, kb = eta c_alpha B_{2 alpha}(0) (c_alpha as in si_kern).
template <typename R, int KT>
struct SiFactor {
  R ka, kb;
  __device__ inline void init(R eta) {
    if constexpr (KT == KT_SI1) {
      ka = eta * (R)19.739208802178716;
      kb = ka * (R)(1.0 / 6.0);
    } else if constexpr (KT == KT_SI2) {
      ka = eta * (R)-64.939394022668291;
      kb = ka * (R)(-1.0 / 30.0);
    } else {
      ka = eta * (R)85.456817206693727;
      kb = ka * (R)(1.0 / 42.0);
    }
  }
  __device__ inline R eta_k(uint32_t u) const {
    const R x = RT<R>::unit(u);
    const R y = fma(x, x, -x);
    if constexpr (KT == KT_SI1) return fma(ka, y, kb);
    else if constexpr (KT == KT_SI2) return fma(ka, y * y, kb);
    else return fma(ka, y * y * (y - (R)0.5), kb);
  }
};

// Derivative sums of the adjoint values u(j) of one column against the
// regenerated column c(j) = gamma prod_q (1 + eta_q K_q(j)):
// acc[q] = sum_j u(j) eta_q dc(j)/d eta_q (product rule over the dimension
// factors), acc[D] = sum_j u(j) c(j).  Padding dimensions carry eta = 0, so
// their factor is exactly 1.
template <typename CR, int KT, int D>
struct LatReduce {
  CR acc[D + 1];
  SiFactor<CR, KT> fk[D];
  CR gam;
  uint32_t u[D], step[D];
  // digits of the thread's first element j0, advanced by step(j_step) per
  // element (padding dimensions: eta = 0, factor exactly 1)
  __device__ inline void init(const uint32_t* __restrict__ gen, const uint32_t* __restrict__ s,
                              int d, const Params* __restrict__ P, uint32_t j0, uint32_t j_step,
                              int m) {
#pragma unroll
    for (int q = 0; q < D; q++) {
      acc[q] = 0;
      fk[q].init(q < d ? RT<CR>::eta(P, q) : (CR)0);
      const uint32_t g = gen[q < d ? q : 0];
      u[q] = lat_z(g, j0, m) + s[q < d ? q : 0];
      step[q] = lat_z(g, j_step, m);
    }
    acc[D] = 0;
    gam = RT<CR>::gamma(P);
  }
  // adds the element at the current digits, then advances them
  __device__ inline void add(CR wv) {
    CR eK[D], f[D], pre[D];
#pragma unroll
    for (int q = 0; q < D; q++) {
      eK[q] = fk[q].eta_k(u[q]);
      f[q] = eK[q] + (CR)1;
      u[q] += step[q];
    }
    CR run = gam * wv;
#pragma unroll
    for (int q = 0; q < D; q++) {
      pre[q] = run;
      run *= f[q];
    }
    acc[D] += run;
    CR suf = 1;
#pragma unroll
    for (int q = D - 1; q >= 0; q--) {
      acc[q] = fma(pre[q] * suf, eK[q], acc[q]);
      suf *= f[q];
    }
  }
  // block sums with one barrier (red: 4 (D + 1) doubles): out[0] = the
  // column sum, out[1 + q] = eta_q sums (q < d), out[1 + d ..] = 0
  __device__ inline void store(int d, double* red, double* out) {
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int q = 0; q <= D; q++) {
      if (q < d || q == D) {
        const double v = wave_sum((double)acc[q]);
        if ((threadIdx.x & 63) == 0) red[w * (D + 1) + q] = v;
      }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < adj_nq(d); q += blockDim.x) {
      double s = 0.0;
      if (q <= d) {
        const int src = q == 0 ? D : q - 1;
        for (int i = 0; i < nw; i++) s += red[i * (D + 1) + src];
      }
      out[q] = s;
    }
  }
};

}  // namespace mtgp

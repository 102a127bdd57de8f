// Many independent fits advanced together: one launch per phase over all
// fits (grouped only by kernel type and dimension width), instead of one
// launch sequence per fit.
//
// Each fit is the loss + gradient of its own plan (Eq. MTGP_MLE_GCV_loss and
// the adjoint of Theorem "Fast MTGP computations"), with sizes n_t <= 2^14,
// so that one workgroup can own a whole kernel column or a whole fit:
//   prep   one workgroup per fit: theta -> Params;
//   fwd    one workgroup per (fit, column): the column generated in natural
//          order and transformed in place through all its index bits
//          (Walsh-Hadamard for nets; radix-2 decimation in frequency for
//          lattices, bit-reversed spectrum) in the fit's FP64 working
//          buffer, a barrier between stages, then stored at the spectrum
//          precision;
//   solve  one workgroup per fit: the fill-free task-order elimination of
//          the unequal-size path (equal sizes are the case n_t / n_u = 1),
//          every stage a barrier apart, with the selected inverse and the
//          adjoint weights written over the spectrum;
//   adj    one workgroup per (fit, column): the transposed transform of the
//          weights (Walsh-Hadamard, or decimation in time from bit-reversed
//          input) and the derivative sums of the regenerated column;
//   final  one workgroup per fit: partial sums and the chain rule;
//   adam   one workgroup per fit.
// The elimination, chain-rule and parameter code is the per-plan path's
// own (elim_dev.h, solve_dev.h), run over a workgroup instead of a grid.
#include <cmath>

#include "elim_dev.h"
#include "fused_eval.h"
#include "latdev.h"
#include "solve_dev.h"

namespace mtgp {

// e^{-i pi k / 2^e} (an exact dyadic angle)
__device__ inline z2 bexpmpi(int64_t k, int e) {
  double s, c;
  sincospi(-ldexp((double)k, -e), &s, &c);
  return {c, s};
}

// Twiddles e^{-i pi q / 2^13}, q < 2^13, as coarse x fine factors (tables of
// 64 and 128 entries in LDS, each factor correctly rounded): the stage of
// bit s < 14 uses q = k 2^(13 - s).
struct BTw {
  z2 hi[64], lo[128];
};
__device__ inline void btw_fill(BTw& tw) {
  for (int q = threadIdx.x; q < 192; q += blockDim.x) {
    if (q < 64) tw.hi[q] = bexpmpi((int64_t)q << 7, 13);
    else tw.lo[q - 64] = bexpmpi(q - 64, 13);
  }
}
__device__ inline z2 btw_at(const BTw& tw, int64_t k, int s) {
  const int q = (int)(k << (13 - s));
  const z2 a = tw.hi[q >> 7], b = tw.lo[q & 127];
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Digits of the points of a digital-sequence column, i = t + 256 k: the
// per-thread part z(t) and, per block, the table z(256 k) XOR shift for the
// k < n / 256 of the column (at most 2^(BATCH_MAX_M - 8) = 64 rows), so that
// u_j(i) = z_j(t) XOR tab[k][j] (z is XOR-linear in the index bits).
template <int D>
struct BDigits {
  uint32_t tab[64][D];
};
template <int D>
__device__ inline void bdigits_fill(BDigits<D>& bd, const uint32_t* gen, const uint32_t* sh, int d,
                                    int m) {
  const int nk = m > 8 ? 1 << (m - 8) : 1;
  for (int q = threadIdx.x; q < nk * D; q += blockDim.x) {
    const int k = q / D, j = q - k * D;
    bd.tab[k][j] = j < d ? dseq_z(gen + 32 * j, (uint32_t)k << 8) ^ sh[j] : 0u;
  }
}

__global__ void batch_prep_kernel(const BFit* __restrict__ fits) {
  const BFit& F = fits[blockIdx.x];
  prep_device(F.theta, F.P, F.kd, F.status);
}

// Pointers read from the fit table are generic to the compiler (flat loads
// and stores, which count against both the vector and the LDS/scalar wait
// counters); they all point to device global memory, and this view of them
// lets the loads and stores of the bodies below be global ones.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ inline gptr<T> glb(T* p) {
  return (gptr<T>)p;
}

// Column c of fit F, FP64, in the fit's working buffer at the column's
// offset (complex interleaved for lattices).
__device__ inline double* bcol_work(const BFit& F, int c) {
  const int64_t off = F.A.col_off[c];
  return F.work + off * (F.kd.family == FAM_LAT ? 2 : 1);
}

// All index bits of one column in place, natural order in.  Nets: the
// unnormalised Walsh-Hadamard transform.  Lattices: radix-2 decimation in
// frequency, X at bit-reversed positions; the stage of bit s multiplies the
// difference by e^{-i pi k / 2^s}, k the index below bit s.
//
// The stages run in rounds of up to 4 bits: a thread loads the 2^R values
// base + q 2^lo (q < 2^R) of a group, applies the round's stages in the
// same order and with the same arithmetic as one stage per pass would, and
// stores them back, so the column crosses the cache once per round, not
// once per bit.  Within a group, the index below bit lo + s is
// k = (base mod 2^lo) + (q mod 2^s) 2^lo.
template <int R, bool FWD>
__device__ __attribute__((always_inline)) inline void block_round(double* w, int m, int lo, bool lat,
                                                                 const BTw& tw) {
  constexpr int Q = 1 << R;
  const int64_t ngroups = ((int64_t)1 << m) >> R;
  const int64_t lo_mask = ((int64_t)1 << lo) - 1;
  for (int64_t g = threadIdx.x; g < ngroups; g += blockDim.x) {
    const int64_t base = (g & lo_mask) | ((g >> lo) << (lo + R));
    const int64_t kb = base & lo_mask;
    if (lat) {
      z2 v[Q];
#pragma unroll
      for (int q = 0; q < Q; q++) {
        const int64_t i = base + ((int64_t)q << lo);
        v[q] = {w[2 * i], w[2 * i + 1]};
      }
#pragma unroll
      for (int r = 0; r < R; r++) {
        const int sb = FWD ? R - 1 - r : r;  // DIF: high bits first; DIT: low first
        const int h = 1 << sb;
#pragma unroll
        for (int q = 0; q < Q; q++) {
          if (q & h) continue;
          const z2 t = btw_at(tw, kb + ((int64_t)(q & (h - 1)) << lo), lo + sb);
          const z2 a = v[q], c = v[q + h];
          if (FWD) {
            const z2 d = {a.x - c.x, a.y - c.y};
            v[q] = {a.x + c.x, a.y + c.y};
            v[q + h] = {d.x * t.x - d.y * t.y, d.x * t.y + d.y * t.x};
          } else {
            const z2 b = {c.x * t.x - c.y * t.y, c.x * t.y + c.y * t.x};
            v[q] = {a.x + b.x, a.y + b.y};
            v[q + h] = {a.x - b.x, a.y - b.y};
          }
        }
      }
#pragma unroll
      for (int q = 0; q < Q; q++) {
        const int64_t i = base + ((int64_t)q << lo);
        w[2 * i] = v[q].x;
        w[2 * i + 1] = v[q].y;
      }
    } else {
      double v[Q];
#pragma unroll
      for (int q = 0; q < Q; q++) v[q] = w[base + ((int64_t)q << lo)];
#pragma unroll
      for (int r = 0; r < R; r++) {
        const int h = 1 << (FWD ? R - 1 - r : r);
#pragma unroll
        for (int q = 0; q < Q; q++) {
          if (q & h) continue;
          const double a = v[q], c = v[q + h];
          v[q] = a + c;
          v[q + h] = a - c;
        }
      }
#pragma unroll
      for (int q = 0; q < Q; q++) w[base + ((int64_t)q << lo)] = v[q];
    }
  }
  __syncthreads();
}

template <bool FWD>
__device__ __attribute__((always_inline)) inline void block_rounds(double* w, int m, bool lat, const BTw& tw) {
  // forward: rounds from the top bits down; adjoint: from bit 0 up
  for (int done = 0; done < m;) {
    const int r = min(4, m - done);
    const int lo = FWD ? m - done - r : done;
    switch (r) {
      case 4: block_round<4, FWD>(w, m, lo, lat, tw); break;
      case 3: block_round<3, FWD>(w, m, lo, lat, tw); break;
      case 2: block_round<2, FWD>(w, m, lo, lat, tw); break;
      default: block_round<1, FWD>(w, m, lo, lat, tw); break;
    }
    done += r;
  }
}
__device__ __attribute__((always_inline)) inline void block_forward(double* w, int m, bool lat,
                                                                   const BTw& tw) {
  block_rounds<true>(w, m, lat, tw);
}
// The transposed network: nets the same Walsh-Hadamard transform;
// lattices decimation in time from bit-reversed input to natural output,
// u(j) = sum_f omega(f) e^{-2 pi i f j / n} with omega(f) at position
// bitrev(f).
__device__ __attribute__((always_inline)) inline void block_adjoint(double* w, int m, bool lat,
                                                                   const BTw& tw) {
  block_rounds<false>(w, m, lat, tw);
}

template <int KT, int D>
__global__ __launch_bounds__(256) void batch_fwd_kernel(const BFit* __restrict__ fits,
                                                        const BItem* __restrict__ items) {
  constexpr int FAM = kt_family(KT);
  __shared__ Kap2Entry k2tab[uses_kap2_table<double, KT>() ? 33 : 1];
  __shared__ BTw tw;  // lattice twiddles
  const BItem it = items[blockIdx.x];
  const BFit& F = fits[it.fit];
  const int c = it.col, d = F.kd.d;
  const int m = F.A.col_m[c];
  const int64_t n = (int64_t)1 << m;
  const Params* P = F.P;
  const uint32_t* sh = F.colshift + (size_t)c * d;
  double* w = bcol_work(F, c);
  if constexpr (uses_kap2_table<double, KT>()) {
    fill_kap2_table(k2tab);
    __syncthreads();
  }
  if constexpr (FAM == FAM_DSEQ) {
    __shared__ BDigits<D> bd;
    bdigits_fill<D>(bd, F.gen, sh, d, m);
    __syncthreads();
    double sc[D];
#pragma unroll
    for (int j = 0; j < D; j++) sc[j] = kscale<double, KT>(j < d ? P->eta[j] : 0.0);
    const double gam = P->gamma;
    Digits<FAM_DSEQ, D> dg;
    dg.init(F.gen, sh, d, threadIdx.x, 0u, m);  // per-thread part z(t)
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      const int k = (int)(i >> 8);
#pragma unroll
      for (int j = 0; j < D; j++) dg.s[j] = bd.tab[k][j];
      double v = gam;
#pragma unroll
      for (int j = 0; j < D; j++) v *= fma(sc[j], kappa_t<double, KT>(dg.u(j), P, k2tab), 1.0);
      w[i] = v;
    }
  } else {
    btw_fill(tw);
    // digits of the thread's first point, advanced by one uniform step per
    // element (natural lattice order); padding dimensions carry eta = 0
    SiFactor<double, KT> fk[D];
    uint32_t u[D], step[D];
#pragma unroll
    for (int q = 0; q < D; q++) {
      fk[q].init(q < d ? P->eta[q] : 0.0);
      const uint32_t g = F.gen[q < d ? q : 0];
      u[q] = lat_z(g, threadIdx.x, m) + sh[q < d ? q : 0];
      step[q] = lat_z(g, blockDim.x, m);
    }
    const double gam = P->gamma;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
      double v = gam;
#pragma unroll
      for (int q = 0; q < D; q++) {
        v = fma(v, fk[q].eta_k(u[q]), v);
        u[q] += step[q];
      }
      w[2 * j] = v;
      w[2 * j + 1] = 0.0;
    }
  }
  __syncthreads();
  block_forward(w, m, FAM == FAM_LAT, tw);
  // spectrum at its storage precision (FP64 fits transform in place)
  const int64_t len = n * (FAM == FAM_LAT ? 2 : 1);
  const int64_t off = F.A.col_off[c] * (FAM == FAM_LAT ? 2 : 1);
  if (F.sr_f32) {
    float* out = static_cast<float*>(F.cols) + off;
    for (int64_t i = threadIdx.x; i < len; i += blockDim.x) out[i] = (float)w[i];
  }
}

// The elimination, stage by stage, all fits per launch: grid (blocks per
// fit, fits[, later tasks]); blocks of a fit that has no such stage exit.
// Each fit's stage runs over the grid-stride range of its blocks, exactly
// as the per-plan launches do.
__device__ inline int64_t bstart() { return blockIdx.x * (int64_t)blockDim.x + threadIdx.x; }
__device__ inline int64_t bstride() { return (int64_t)gridDim.x * blockDim.x; }
__device__ inline z2* bz_rr(const BFit& F) { return F.S + F.A.so[F.A.T]; }
__device__ inline z2* bz_U(const BFit& F) { return F.S + F.A.so[F.A.T] + F.N; }

__global__ __launch_bounds__(256) void batch_zf_init_kernel(const BFit* __restrict__ fits) {
  const BFit& F = fits[blockIdx.y];
  const gptr<const Params> P = glb((const Params*)F.P);
  const gptr<const double> yhat = glb((const double*)F.yhat);
  const gptr<z2> S = glb(F.S), rr = glb(bz_rr(F)), U = glb(bz_U(F));
  if (F.sr_f32)
    zf_init_body<float>(glb(static_cast<const float*>(F.cols)), F.A, P, F.kd.family, F.N, yhat, S,
                        rr, U, bstart(), bstride());
  else
    zf_init_body<double>(glb(static_cast<const double*>(F.cols)), F.A, P, F.kd.family, F.N, yhat,
                         S, rr, U, bstart(), bstride());
}

// stage t, later task u = t + 1 + blockIdx.z (the targets of different u
// are independent)
__global__ __launch_bounds__(256) void batch_zf_factor_kernel(const BFit* __restrict__ fits, int t) {
  const BFit& F = fits[blockIdx.y];
  const int u = t + 1 + (int)blockIdx.z;
  if (u >= F.A.T) return;
  const int64_t K = 1ll << (F.A.m[t] - F.A.m[u]);
  const int G = K >= 64 ? 64 : (int)K;
  zf_factor_body(F.A, t, u, G, glb(F.S), glb(bz_rr(F)), glb(bz_U(F)), bstart(), bstride());
}

// backward stage k of every fit: its task T - 1 - k
__global__ __launch_bounds__(256) void batch_zf_back_kernel(const BFit* __restrict__ fits, int k) {
  const BFit& F = fits[blockIdx.y];
  const int T = F.A.T, t = T - 1 - k;
  if (t < 0) return;
  const gptr<z2> S = glb(F.S), rr = glb(bz_rr(F)), U = glb(bz_U(F));
  const gptr<double> logs = glb(F.logs);
  const gptr<int> status = glb(F.status);
  if (T <= 1) zf_back_body<1, true>(F.A, t, S, rr, U, logs, status, bstart(), bstride());
  else if (T <= 2) zf_back_body<2, true>(F.A, t, S, rr, U, logs, status, bstart(), bstride());
  else if (T <= 4) zf_back_body<4, true>(F.A, t, S, rr, U, logs, status, bstart(), bstride());
  else if (T <= 8) zf_back_body<8, true>(F.A, t, S, rr, U, logs, status, bstart(), bstride());
  else zf_back_body<16, true>(F.A, t, S, rr, U, logs, status, bstart(), bstride());
}

__global__ __launch_bounds__(256) void batch_zf_tau_kernel(const BFit* __restrict__ fits) {
  const BFit& F = fits[blockIdx.x];
  zf_tau_body(F.A, F.P, bz_rr(F), bz_U(F));
}

template <typename SR>
__device__ inline void bz_final(const BFit& F) {
  const gptr<SR> cols = glb(static_cast<SR*>(F.cols));
  const int T = F.A.T;
  const gptr<z2> S = glb(F.S), rr = glb(bz_rr(F)), U = glb(bz_U(F));
  // partial row of this block; the row layout of the chain rule: TM = solve_tm(T)
  double* row = F.sp + (size_t)blockIdx.x * solve_ns(T);
#define MTGP_BZF(TMV)                                                                          \
  zf_final_body<SR, TMV>(cols, F.A, F.N, glb((const Params*)F.P), F.kd.family, 1,                \
                         glb((const double*)F.yhat), S, rr, U, nullptr, row,                    \
                         bstart(), bstride())
  if (T <= 1) MTGP_BZF(1);
  else if (T <= 2) MTGP_BZF(2);
  else if (T <= 4) MTGP_BZF(4);
  else if (T <= 8) MTGP_BZF(8);
  else MTGP_BZF(16);
#undef MTGP_BZF
}

__global__ __launch_bounds__(256) void batch_zf_final_kernel(const BFit* __restrict__ fits) {
  const BFit& F = fits[blockIdx.y];
  if (F.sr_f32) bz_final<float>(F);
  else bz_final<double>(F);
}

template <int KT, int D>
__global__ __launch_bounds__(256) void batch_adj_kernel(const BFit* __restrict__ fits,
                                                        const BItem* __restrict__ items) {
  constexpr int FAM = kt_family(KT);
  constexpr bool ADAPT = KT == KT_DSIA;
  constexpr int NQ = D + 5;
  __shared__ Kap2Entry k2tab[uses_kap2_table<double, KT>() ? 33 : 1];
  __shared__ double red[4 * NQ];
  const BItem it = items[blockIdx.x];
  const BFit& F = fits[it.fit];
  const int c = it.col, d = F.kd.d;
  const int m = F.A.col_m[c];
  const int64_t n = (int64_t)1 << m;
  const Params* P = F.P;
  const uint32_t* sh = F.colshift + (size_t)c * d;
  double* w = bcol_work(F, c);
  const int nq = adj_nq(d);
  double* out = F.ap + (size_t)c * nq;
  // the weights at FP64 in the working buffer
  const int64_t len = n * (FAM == FAM_LAT ? 2 : 1);
  const int64_t off = F.A.col_off[c] * (FAM == FAM_LAT ? 2 : 1);
  if (F.sr_f32) {
    const float* in = static_cast<const float*>(F.cols) + off;
    for (int64_t i = threadIdx.x; i < len; i += blockDim.x) w[i] = (double)in[i];
  }
  if constexpr (uses_kap2_table<double, KT>()) fill_kap2_table(k2tab);
  __shared__ BTw tw;
  __shared__ BDigits<FAM == FAM_DSEQ ? D : 1> bd;
  if constexpr (FAM == FAM_LAT) btw_fill(tw);
  else bdigits_fill<D>(bd, F.gen, sh, d, m);
  __syncthreads();
  block_adjoint(w, m, FAM == FAM_LAT, tw);
  if constexpr (FAM == FAM_DSEQ) {
    double acc[D + 1];
    double acc_b[4] = {0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j <= D; j++) acc[j] = 0;
    double sc[D];
#pragma unroll
    for (int j = 0; j < D; j++) sc[j] = kscale<double, KT>(j < d ? P->eta[j] : 0.0);
    const double gam = P->gamma;
    Digits<FAM_DSEQ, D> dg;
    dg.init(F.gen, sh, d, threadIdx.x, 0u, m);  // per-thread part z(t)
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      const int k = (int)(i >> 8);
#pragma unroll
      for (int j = 0; j < D; j++) dg.s[j] = bd.tab[k][j];
      adj_element<double, KT, D>(dg, w[i], gam, sc, P, k2tab, acc, acc_b);
    }
#pragma unroll
    for (int j = 0; j < D; j++) acc[j] *= sc[j];
    // block sums; row layout [0] w c, [1..d] eta_j, [d+1..d+4] b_alpha
    const int wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NQ; q++) {
      const bool used = q < D ? q < d : (q == D || ADAPT);
      if (used) {
        const double v = wave_sum(q <= D ? acc[q < D ? q : D] : acc_b[q - D - 1]);
        if ((threadIdx.x & 63) == 0) red[wv * NQ + q] = v;
      }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < nq; q += blockDim.x) {
      const int src = q == 0 ? D : (q <= d ? q - 1 : D + 1 + (q - d - 1));
      double s = 0.0;
      if (src < D + 1 || ADAPT)
        for (int i = 0; i < nw; i++) s += red[i * NQ + src];
      out[q] = s;
    }
  } else {
    LatReduce<double, KT, D> lr;
    lr.init(F.gen, sh, d, P, (uint32_t)threadIdx.x, (uint32_t)blockDim.x, m);
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) lr.add(w[2 * j]);
    lr.store(d, red, out);
  }
}

__global__ __launch_bounds__(256) void batch_final_kernel(const BFit* __restrict__ fits) {
  const BFit& F = fits[blockIdx.x];
  // log det = the sum of the log pivots
  finalize_device(F.sp, BATCH_SOLVE_BLOCKS, F.ap, F.colinfo, F.ncol, F.logs, (int)F.N, F.yhat,
                  (int64_t)1 << F.kd.m[0], F.P, F.kd, F.out3, F.grad, nullptr);
}

__global__ __launch_bounds__(256) void batch_adam_kernel(const BFit* __restrict__ fits, double lr,
                                                         double b1, double b2, double eps) {
  const BFit& F = fits[blockIdx.x];
  const int64_t k = *F.step + 1;
  const double c1 = 1.0 - pow(b1, (double)k), c2 = 1.0 - pow(b2, (double)k);
  double* theta = const_cast<double*>(F.theta);
  for (int64_t i = threadIdx.x; i < F.ntheta; i += blockDim.x) {
    if (F.frozen && F.frozen[i]) continue;
    const double g = F.grad[i];
    const double a = b1 * F.m1[i] + (1.0 - b1) * g;
    const double b = b2 * F.m2[i] + (1.0 - b2) * g * g;
    F.m1[i] = a;
    F.m2[i] = b;
    theta[i] -= lr * (a / c1) / (sqrt(b / c2) + eps);
  }
  __syncthreads();
  if (threadIdx.x == 0) *F.step = k;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int launch_batch_prep(const BFit* fits, int nfits, hipStream_t st) {
  if (nfits <= 0) return 0;
  hipLaunchKernelGGL(batch_prep_kernel, dim3(nfits), dim3(64), 0, st, fits);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_batch_solve(const BFit* fits, int nfits, int tmax, hipStream_t st) {
  if (nfits <= 0) return 0;
  const dim3 grid(BATCH_SOLVE_BLOCKS, (unsigned)nfits), block(256);
  hipLaunchKernelGGL(batch_zf_init_kernel, grid, block, 0, st, fits);
  for (int t = 0; t + 1 < tmax; t++)
    hipLaunchKernelGGL(batch_zf_factor_kernel, dim3(BATCH_SOLVE_BLOCKS, (unsigned)nfits,
                                                    (unsigned)(tmax - 1 - t)),
                       block, 0, st, fits, t);
  for (int k = 0; k < tmax; k++)
    hipLaunchKernelGGL(batch_zf_back_kernel, grid, block, 0, st, fits, k);
  hipLaunchKernelGGL(batch_zf_tau_kernel, dim3((unsigned)nfits), block, 0, st, fits);
  hipLaunchKernelGGL(batch_zf_final_kernel, grid, block, 0, st, fits);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_batch_final(const BFit* fits, int nfits, hipStream_t st) {
  if (nfits <= 0) return 0;
  hipLaunchKernelGGL(batch_final_kernel, dim3(nfits), dim3(256), 0, st, fits);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_batch_adam(const BFit* fits, int nfits, double lr, double b1, double b2, double eps,
                      hipStream_t st) {
  if (nfits <= 0) return 0;
  hipLaunchKernelGGL(batch_adam_kernel, dim3(nfits), dim3(256), 0, st, fits, lr, b1, b2, eps);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int KT>
static void fwd_kt(const BFit* fits, const BItem* items, int nitems, int d, hipStream_t st) {
#define MTGP_BF(DD, KTV) \
  hipLaunchKernelGGL((batch_fwd_kernel<KTV, DD>), dim3(nitems), dim3(256), 0, st, fits, items)
  MTGP_DISPATCH_D(d, MTGP_BF, KT);
#undef MTGP_BF
}

template <int KT>
static void adj_kt(const BFit* fits, const BItem* items, int nitems, int d, hipStream_t st) {
#define MTGP_BA(DD, KTV) \
  hipLaunchKernelGGL((batch_adj_kernel<KTV, DD>), dim3(nitems), dim3(256), 0, st, fits, items)
  MTGP_DISPATCH_D(d, MTGP_BA, KT);
#undef MTGP_BA
}

#define MTGP_BATCH_KT_SWITCH(FN)                          \
  switch (kt) {                                           \
    case KT_DSI1: FN<KT_DSI1>(fits, items, nitems, d, st); break; \
    case KT_DSI2: FN<KT_DSI2>(fits, items, nitems, d, st); break; \
    case KT_DSI3: FN<KT_DSI3>(fits, items, nitems, d, st); break; \
    case KT_DSI4: FN<KT_DSI4>(fits, items, nitems, d, st); break; \
    case KT_DSIA: FN<KT_DSIA>(fits, items, nitems, d, st); break; \
    case KT_SI1: FN<KT_SI1>(fits, items, nitems, d, st); break;   \
    case KT_SI2: FN<KT_SI2>(fits, items, nitems, d, st); break;   \
    case KT_SI3: FN<KT_SI3>(fits, items, nitems, d, st); break;   \
    default: return -1;                                   \
  }

int launch_batch_fwd(const BFit* fits, const BItem* items, int nitems, int kt, int d,
                     hipStream_t st) {
  if (nitems <= 0) return 0;
  MTGP_BATCH_KT_SWITCH(fwd_kt)
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_batch_adj(const BFit* fits, const BItem* items, int nitems, int kt, int d,
                     hipStream_t st) {
  if (nitems <= 0) return 0;
  MTGP_BATCH_KT_SWITCH(adj_kt)
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
#undef MTGP_BATCH_KT_SWITCH

}  // namespace mtgp

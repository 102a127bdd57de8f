// Fused kernel-column evaluation kernels of the digital-sequence path, one
// translation unit per kernel order (fused_o*.hip instantiate them):
//
//   gen_fwd_kernel    column generation fused with the low-bit (LDS) forward
//                     Walsh-Hadamard pass: raw columns never reach HBM;
//   adj_reduce_kernel the low-bit adjoint pass fused with the derivative
//                     reduction of the regenerated columns.
//
// Dimension slots are padded to the template width D with eta = 0, so the
// padding factors are exactly 1 and the loops carry no run-time guards.  With
// a 2^12-point LDS block (E = 16 elements per thread) the generation kernel
// transforms the index bits 8 .. 11 in registers and only bits 0 .. 7 in LDS.
#pragma once
#include "colgen.h"

namespace mtgp {

// ---------------------------------------------------------------------------
// pass A fused with column generation (digital sequences): grid (2^(m-LB), ncols)
// arithmetic in Real, block stored as TOut
// ---------------------------------------------------------------------------
template <typename Real, typename TOut, int KT, int D, int E>
__global__ __launch_bounds__(256) void gen_fwd_kernel(TOut* __restrict__ base, int64_t col_stride,
                                                      int m, int LB, int G,
                                                      const uint32_t* __restrict__ gen,
                                                      const uint32_t* __restrict__ colshift,
                                                      const Params* __restrict__ P, int d) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ Kap2Entry k2tab[uses_kap2_table<Real, KT>() ? 33 : 1];
  Real* lds = reinterpret_cast<Real*>(smem);
  const int nb = 1 << LB;
  const int col = blockIdx.y;
  const uint32_t t = threadIdx.x;
  const int stride = lds_stride(LB);
  const uint32_t* cs = colshift + (size_t)col * d;
  if constexpr (uses_kap2_table<Real, KT>()) {
    fill_kap2_table(k2tab);
    __syncthreads();
  }
  Digits<FAM_DSEQ, D> dg;   // blocks below 256 E points (E = 0)
  FoldedDigits<D> fd;       // E > 0
  const uint32_t* gz = gray_table(gen, d);
  Real sc[D];  // eta K = sc kappa; padding slots: sc = 0, factor exactly 1
#pragma unroll
  for (int j = 0; j < D; j++) sc[j] = kscale<Real, KT>(j < d ? RT<Real>::eta(P, j) : (Real)0);
  const Real gam = RT<Real>::gamma(P);
  // G consecutive blocks of the column per workgroup: the per-thread digit
  // parts and the table are set up once for all of them
  for (int g = 0; g < G; g++) {
    const uint32_t i0 = ((uint32_t)blockIdx.x * G + g) << LB;
    if (g > 0) __syncthreads();  // the previous block's stores have read the tile
    if constexpr (E > 0) {
      // nb == 256 E: thread t owns indices t + 256 e.  Index bits 8 .. 8+log2(E)
      // are transformed in registers, bits 0 .. 7 in two LDS rounds.
      Real v[E];
      if (g == 0) fd.init(gen, cs, d, t, i0);
      else fd.set_block(gen, d, i0 - (1u << LB), i0);
      fd.ahead(gz);
#pragma unroll
      for (int k = 0; k < E; k++) {
        if (k > 0) fd.step(gz, k);
        Real c = gam;
#pragma unroll
        for (int j = 0; j < D; j++) c *= fma(sc[j], kappa_t<Real, KT>(fd.u(j), P, k2tab), (Real)1);
        v[Digits<FAM_DSEQ, D>::elem(k)] = c;
        fd.hold_rows();
      }
      reg_fwht<Real, E>(v);
#pragma unroll
      for (int k = 0; k < E; k++) lds[lds_at(0, stride, (int)t + 256 * k)] = v[k];
      __syncthreads();
      lds_round<Real, 4>(lds, 1, LB, 0, stride);
      __syncthreads();
      lds_round<Real, 4>(lds, 1, LB, 4, stride);
      __syncthreads();
    } else {
      const int En = nb > 256 ? nb >> 8 : 1;
      if ((int)t < nb) {
        if (g == 0) dg.init(gen, cs, d, t, i0, m);
        else dg.set_block(gen, cs, d, i0, m);
        for (int k = 0; k < En; k++) {
          Real c = gam;
#pragma unroll
          for (int j = 0; j < D; j++) c *= fma(sc[j], kappa_t<Real, KT>(dg.u(j), P, k2tab), (Real)1);
          lds[lds_at(0, stride, (int)t + 256 * dg.elem(k))] = c;
          if (k + 1 < En) dg.advance(gen, d, k);
        }
      }
      lds_fwht<Real>(lds, 1, LB, stride);
    }
    TOut* out = base + (size_t)col * col_stride + i0;
    for (int e = t; e < nb; e += 256) out[e] = (TOut)lds[lds_at(0, stride, e)];
  }
}

// ---------------------------------------------------------------------------
// Adjoint pass: low-bit Walsh-Hadamard stages of the adjoint weights fused
// with the derivative reduction of the kernel columns.
//
// With Ktilde = V Lambda V^dagger and V independent of theta,
//   dL/dtheta = sum_f trace(W(f) dLambda(f)),  W = Lambda^-1 - ahat ahat^dagger
// (ahat = Lambda^-1 rhat).  Lambda's entries are R_tu times transforms of
// kernel columns c_p, so the column part of the gradient is
//   sum_p sum_i w_p(i) dc_p(i)/dtheta,  w_p = (transform of omega_p)
// where omega_p collects R-weighted W entries of every pair using column p
// (solve kernel).  adj_reduce_kernel finishes the transform of omega_p over the low
// index bits, regenerates c_p's factors in registers and accumulates
//   dc/dlog eta_j = gamma eta_j K_j prod_{k != j} (1 + eta_k K_k)
// with prefix / suffix products (no division: a factor 1 + eta K may be 0),
// plus dc/dlog b_alpha for the adaptive kernel and c itself (dc/dlog gamma).
// ---------------------------------------------------------------------------

// Accumulates the derivative sums of one element with weight wv: slot j
// gets w gamma kappa_j prod_{k != j} f_k (times sc_j at the end this is
// w dc/dlog eta_j), slot D gets w c, acc_b the adaptive-weight sums.
template <typename Real, int KT, int D, typename Dg>
__device__ inline void adj_element(const Dg& dg, Real wv, Real gam,
                                   const Real (&sc)[D], const Params* __restrict__ P,
                                   const Kap2Entry* k2tab, Real (&acc)[D + 1],
                                   Real (&acc_b)[4]) {
  constexpr bool ADAPT = KT == KT_DSIA;
  Real kap[D], f[D];
  Real Ka[ADAPT ? D : 1][4];
#pragma unroll
  for (int j = 0; j < D; j++) {
    if constexpr (ADAPT) {
      dsi_khat_all<Real>(dg.u(j), Ka[j]);
      kap[j] = RT<Real>::bw(P, 0) * Ka[j][0] + RT<Real>::bw(P, 1) * Ka[j][1] +
               RT<Real>::bw(P, 2) * Ka[j][2] + RT<Real>::bw(P, 3) * Ka[j][3];
    } else {
      kap[j] = kappa_t<Real, KT>(dg.u(j), P, k2tab);
    }
    f[j] = fma(sc[j], kap[j], (Real)1);
  }
  // pre[j] = w gamma prod_{k<j} f_k; the suffix product runs backwards
  Real pre[D];
  Real run = gam * wv;
#pragma unroll
  for (int j = 0; j < D; j++) {
    pre[j] = run;
    run *= f[j];
  }
  acc[D] += run;  // w * c
  Real suf = 1;
#pragma unroll
  for (int j = D - 1; j >= 0; j--) {
    const Real ps = pre[j] * suf;  // w gamma prod_{k != j} f_k
    acc[j] = fma(ps, kap[j], acc[j]);
    if constexpr (ADAPT) {
      const Real pe = ps * sc[j];
#pragma unroll
      for (int q = 0; q < 4; q++) acc_b[q] = fma(pe, Ka[j][q], acc_b[q]);
    }
    suf *= f[j];
  }
}

// run != 0: the weights are in the run layout with the halves of the row
// index swapped (as the one-pass adjoint transform writes them, 4096 rows):
// block h's element e sits at run_index(run_swap(h), e), so each 16-element
// segment is one 128-byte line.
template <typename Real, typename TIn, int KT, int D>
__global__ __launch_bounds__(256) void adj_reduce_kernel(const TIn* __restrict__ base,
                                                         int64_t col_stride, int m, int LB, int G,
                                                         const uint32_t* __restrict__ gen,
                                                         const uint32_t* __restrict__ colshift,
                                                         const Params* __restrict__ P, int d,
                                                         double* __restrict__ partials, int run) {
  constexpr int FAM = kt_family(KT);
  constexpr bool ADAPT = KT == KT_DSIA;
  constexpr int NQ = D + 5;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[4 * NQ];
  __shared__ Kap2Entry k2tab[uses_kap2_table<Real, KT>() ? 33 : 1];
  Real* lds = reinterpret_cast<Real*>(smem);
  const int nb = 1 << LB;
  const int col = blockIdx.y;
  const uint32_t t = threadIdx.x;
  const int stride = lds_stride(LB);
  const uint32_t* cs = colshift + (size_t)col * d;
  // the barriers of the transform below order the table's fill before its use
  if constexpr (uses_kap2_table<Real, KT>()) fill_kap2_table(k2tab);
  Real acc[D + 1];
  Real acc_b[4] = {0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j <= D; j++) acc[j] = 0;
  Real sc[D];  // eta K = sc kappa; padding slots: sc = 0
#pragma unroll
  for (int j = 0; j < D; j++) sc[j] = kscale<Real, KT>(j < d ? RT<Real>::eta(P, j) : (Real)0);
  const Real gam = RT<Real>::gamma(P);
  static_assert(FAM == FAM_DSEQ, "digital-sequence kernels only");
  FoldedDigits<D> dg;
  const uint32_t* gz = gray_table(gen, d);
  // LDS slot of element t + 256 e: lds_at(0, stride, t + 256 e) = wb + 272 e
  const int wb = (int)t + ((int)t >> 4);
  // the element loop stays rolled: unrolled, its per-element temporaries
  // exceed the register file
  const int En = nb > 256 ? nb >> 8 : 1;
  // G consecutive blocks of the column per workgroup: the per-thread digit
  // parts and the block reduction below are paid once for all of them
  const TIn* colp = base + (size_t)col * col_stride;
  uint32_t i0_prev = 0;
  for (int g = 0; g < G; g++) {
    const int h = (int)blockIdx.x * G + g;
    const uint32_t i0 = (uint32_t)h << LB;
    // block h's element e: natural colp[i0 + e], runs colp[run_index(run_swap(h), e)]
    const TIn* w = run ? colp + ((int64_t)run_swap(h) << 4) : colp + i0;
    if (g > 0) __syncthreads();  // every read of the previous block's tile is done
    if (LB == 12) {
      // 16 loads in flight per thread, index bits 8 .. 11 in registers, bits
      // 0 .. 7 in two LDS rounds
      Real v[16];
      if (run) {
        // e = t + 256 k: run_index offset ((t >> 4) + 16 k) 2^16 + (t & 15)
        const TIn* wt = w + ((int64_t)(t >> 4) << 16) + (t & 15);
#pragma unroll
        for (int k = 0; k < 16; k++) v[k] = (Real)wt[(int64_t)k << 20];
      } else {
#pragma unroll
        for (int k = 0; k < 16; k++) v[k] = (Real)w[t + 256 * k];
      }
      reg_fwht<Real, 16>(v);
#pragma unroll
      for (int k = 0; k < 16; k++) lds[lds_at(0, stride, (int)t + 256 * k)] = v[k];
      __syncthreads();
      lds_round<Real, 4>(lds, 1, LB, 0, stride);
      __syncthreads();
      lds_round<Real, 4>(lds, 1, LB, 4, stride);
      __syncthreads();
    } else {
      for (int i = threadIdx.x; i < nb; i += blockDim.x)
        lds[lds_at(0, stride, i)] =
            (Real)(run ? w[((int64_t)(i >> 4) << 16) + (i & 15)] : w[i]);
      lds_fwht<Real>(lds, 1, LB, stride);
    }
    if ((int)t < nb) {
      if (g == 0) dg.init(gen, cs, d, t, i0);
      else dg.set_block(gen, d, i0_prev, i0);
      dg.ahead(gz);
      for (int k = 0; k < En; k++) {
        if (k > 0) dg.step(gz, k);
        const Real wv = lds[wb + 272 * Digits<FAM_DSEQ, D>::elem(k)];
        adj_element<Real, KT, D>(dg, wv, gam, sc, P, k2tab, acc, acc_b);
        dg.hold();
      }
    }
    i0_prev = i0;
  }
  if ((int)t < nb) {
#pragma unroll
    for (int j = 0; j < D; j++) acc[j] *= sc[j];  // kappa sums -> dc/dlog eta_j sums
  }
  // block sums, one barrier; slot layout [eta_0 .. eta_{D-1}, c, b_0 .. b_3]
  const int wv_id = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    const bool used = q < D ? q < d : (q == D || ADAPT);
    if (used) {
      const double v = wave_sum(q <= D ? (double)acc[q < D ? q : D] : (double)acc_b[q - D - 1]);
      if ((threadIdx.x & 63) == 0) red[wv_id * NQ + q] = v;
    }
  }
  __syncthreads();
  // output layout: [0] w c (gamma), [1..d] eta_j, [d+1..d+4] b_alpha (without the b factor)
  const int nq = adj_nq(d);
  double* out = partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * nq;
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    const int src = q == 0 ? D : (q <= d ? q - 1 : D + 1 + (q - d - 1));
    double s = 0.0;
    if (src < D + 1 || ADAPT)
      for (int i = 0; i < nw; i++) s += red[i * NQ + src];
    out[q] = s;
  }
}

// ---------------------------------------------------------------------------
// launchers (one kernel type; dimension width and block shape dispatched here)
// ---------------------------------------------------------------------------
template <typename Real, int KT>
constexpr bool fused_reg_stages() {
  // register stages for the FP64-arithmetic paths of the fixed-order kernels
  return sizeof(Real) == 8 && KT != KT_DSIA;
}

template <typename Real, typename TOut, int KT, int D>
void gen_fwd_launch_d(dim3 grid, size_t lds, hipStream_t st, bool regs, int G, TOut* base,
                      int64_t col_stride, int m, int LB, const uint32_t* gen,
                      const uint32_t* colshift, const Params* P, int d) {
  if constexpr (fused_reg_stages<Real, KT>()) {
    if (regs) {
      hipLaunchKernelGGL((gen_fwd_kernel<Real, TOut, KT, D, 16>), grid, dim3(256), lds, st, base,
                         col_stride, m, LB, G, gen, colshift, P, d);
      return;
    }
  }
  hipLaunchKernelGGL((gen_fwd_kernel<Real, TOut, KT, D, 0>), grid, dim3(256), lds, st, base,
                     col_stride, m, LB, G, gen, colshift, P, d);
}

template <typename Real, typename TOut, int KT>
int launch_gen_fwd_kt(TOut* base, int64_t col_stride, int ncols, int m, const uint32_t* gen,
                      const uint32_t* colshift, const Params* P, int d, const Sched& sc,
                      hipStream_t st) {
  const int LB = sc.lb(m);
  const size_t lds = sc.fused_lds(gen_cols_lds_bytes(LB, sizeof(Real)));
  const int64_t nblk = (int64_t)1 << (m - LB);
  const int G = gen_group(nblk);
  const dim3 grid((unsigned)(nblk / G), (unsigned)ncols);
  const bool regs = LB == 12;
#define MTGP_GEN(DD, KTV) \
  gen_fwd_launch_d<Real, TOut, KTV, DD>(grid, lds, st, regs, G, base, col_stride, m, LB, gen, \
                                        colshift, P, d)
  MTGP_DISPATCH_D(d, MTGP_GEN, KT);
#undef MTGP_GEN
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename Real, typename TIn, int KT>
int launch_adj_reduce_kt(const TIn* base, int64_t col_stride, int ncols, int m,
                         const uint32_t* gen, const uint32_t* colshift, const Params* P, int d,
                         double* partials, const Sched& sc, hipStream_t st, int run) {
  const int LB = sc.lb(m);
  const size_t lds = sc.fused_lds(gen_cols_lds_bytes(LB, sizeof(Real)));
  const int64_t nblk = (int64_t)1 << (m - LB);
  const int G = adj_group(nblk);
  // the run layout holds 4096 rows of 16-index groups
  if (run && (nblk != 4096 || LB < 4)) return -1;
  const dim3 grid((unsigned)(nblk / G), (unsigned)ncols);
#define MTGP_ADJ(DD, KTV)                                                                        \
  hipLaunchKernelGGL((adj_reduce_kernel<Real, TIn, KTV, DD>), grid, dim3(256), lds, st, base,     \
                     col_stride, m, LB, G, gen, colshift, P, d, partials, run)
  MTGP_DISPATCH_D(d, MTGP_ADJ, KT);
#undef MTGP_ADJ
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace mtgp

// Shifted rank-1 lattices with shift-invariant kernels (Condition "Fast
// MTGP", SI-LAT): V^dagger a = n^-1/2 F (bit reversal of a) (Theorem "Fast
// GP computations"), so kernel columns are taken in natural lattice order
// j (point j g / n + shift) and transformed by the unnormalised DFT
// F_fj = e^{-2 pi i f j / n}.
//
// Four-step split n = n1 n2, j = j1 + n1 j2, f = f2 + n2 f1 (n1 <= 2^12):
//   pass 1 (strided, fused with column generation or the bit-reversed data
//           load): for each j1, DFT over j2, twiddle e^{-2 pi i f2 j1 / n},
//           store Y[f2][j1]  (tiles of KC consecutive j1: wide segments);
//   pass 2 (contiguous): for each f2, DFT over j1, store X[f2][f1].
// The spectrum therefore lives at position p = f2 n1 + f1 for frequency
// f = f2 + n2 f1; the per-frequency algebra does not care about the order,
// and the data transform uses the same layout.  Frequency 0 sits at p = 0.
// The adjoint u(j) = Re sum_f omega(f) e^{-2 pi i f j / n} runs the mirror
// image: pass A' (contiguous over f1, twiddle e^{-2 pi i j1 f2 / n}) and
// pass B' (strided over f2) fused with the derivative reduction.
// Each in-LDS DFT is radix-2 decimation in frequency (natural input,
// bit-reversed output) with a per-block twiddle table.
#include "colgen.h"

namespace mtgp {

template <typename R>
__device__ inline cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// e^{-2 pi i k / 2^bits} for 0 <= k < 2^bits, FP64 (the angle is an exact dyadic)
__device__ inline cx<double> twiddle64(int64_t k, int bits) {
  double s, c;
  sincospi(-ldexp((double)k, 1 - bits), &s, &c);
  return {c, s};
}

// In-LDS radix-2 DIF DFT of nseq sequences of length 2^L; afterwards position
// p holds frequency bitrev_L(p).  tw[k] = e^{-2 pi i k / 2^L}, k < 2^(L-1).
template <typename R>
__device__ inline void lds_fft(cx<R>* a, int nseq, int L, int stride, const cx<R>* tw) {
  if (L == 0) {
    __syncthreads();
    return;
  }
  const int hb = L - 1;
  const int total = nseq << hb;
  for (int s = L - 1; s >= 0; s--) {
    __syncthreads();
    const int half = 1 << s;
    for (int g = threadIdx.x; g < total; g += blockDim.x) {
      const int seq = g >> hb;
      const int q = g & ((1 << hb) - 1);
      const int k = q & (half - 1);
      const int i = ((q >> s) << (s + 1)) | k;
      cx<R>* pa = a + lds_at(seq, stride, i);
      cx<R>* pb = a + lds_at(seq, stride, i + half);
      const cx<R> A = *pa, B = *pb;
      *pa = {A.x + B.x, A.y + B.y};
      *pb = cmul<R>({A.x - B.x, A.y - B.y}, tw[k << (hb - s)]);
    }
  }
  __syncthreads();
}

__device__ inline int bitrev_bits(int p, int L) { return L ? (int)(__brev((uint32_t)p) >> (32 - L)) : 0; }

template <typename R>
__device__ inline void fill_twiddles(cx<R>* tw, int L) {
  for (int k = threadIdx.x; k < (L ? (1 << (L - 1)) : 0); k += blockDim.x) {
    const cx<double> w = twiddle64(k, L);
    tw[k] = {(R)w.x, (R)w.y};
  }
}

// lattice kernel column value at natural index j of a column with shift sh
template <typename R, int KT>
__device__ inline R lat_col_value(const uint32_t* __restrict__ gen, const uint32_t* __restrict__ sh,
                                  int d, uint32_t j, int m, const Params* __restrict__ P) {
  R c = RT<R>::gamma(P);
  for (int q = 0; q < d; q++)
    c = fma(c * RT<R>::eta(P, q), kval<R, KT>(lat_z(gen[q], j, m) + sh[q], P), c);
  return c;
}

enum { SRC_GEN = LAT_SRC_GEN, SRC_Y = LAT_SRC_Y, SRC_X = LAT_SRC_X };

// data value at natural index j of vector v: y[bitrev_m(j)] (SRC_Y) or y[j] (SRC_X)
__device__ inline double load_data(const void* y, int y_f32, int src, int v, uint32_t j, int m) {
  const size_t idx = (size_t)v * ((size_t)1 << m) + (src == SRC_Y ? (uint32_t)bitrev_bits((int)j, m) : j);
  return y_f32 ? (double)static_cast<const float*>(y)[idx] : static_cast<const double*>(y)[idx];
}

// Pass 1: tile = KC consecutive j1 x n2 rows; grid (n1 / KC, nvec).
// SRC_GEN: value = kernel column c(j); SRC_Y: value = y[bitrev_m(j)] of vector v.
template <typename CR, int SRC, int KT>
__global__ __launch_bounds__(256) void lat_pass1_kernel(cx<CR>* __restrict__ Y, int64_t vstride,
                                                        const void* __restrict__ y, int y_f32, int m,
                                                        int b1, int KC,
                                                        const uint32_t* __restrict__ gen,
                                                        const uint32_t* __restrict__ colshift,
                                                        const Params* __restrict__ P, int d) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b2 = m - b1, n1 = 1 << b1, n2 = 1 << b2;
  const int stride = lds_stride(b2);
  cx<CR>* a = reinterpret_cast<cx<CR>*>(smem);
  cx<CR>* tw = a + (size_t)KC * stride;
  const int v = blockIdx.y;
  const int j1_0 = blockIdx.x * KC;
  fill_twiddles<CR>(tw, b2);
  const int kcb = __ffs(KC) - 1;
  for (int q = threadIdx.x; q < (KC << b2); q += blockDim.x) {
    const int kc = q & (KC - 1), j2 = q >> kcb;
    const uint32_t j = (uint32_t)(j1_0 + kc) + ((uint32_t)j2 << b1);
    CR val;
    if (SRC == SRC_GEN)
      val = lat_col_value<CR, KT>(gen, colshift + (size_t)v * d, d, j, m, P);
    else
      val = (CR)load_data(y, y_f32, SRC, v, j, m);
    a[lds_at(kc, stride, j2)] = {val, (CR)0};
  }
  lds_fft<CR>(a, KC, b2, stride, tw);
  cx<CR>* out = Y + (size_t)v * vstride;
  for (int q = threadIdx.x; q < (KC << b2); q += blockDim.x) {
    const int kc = q & (KC - 1), f2 = q >> kcb;
    const int j1 = j1_0 + kc;
    const cx<CR> val = a[lds_at(kc, stride, bitrev_bits(f2, b2))];
    const cx<double> w = twiddle64((int64_t)f2 * j1, m);
    out[(size_t)f2 * n1 + j1] = cmul<CR>(val, {(CR)w.x, (CR)w.y});
  }
  (void)n2;
}

// Pass 2: one block per row f2 (grid (n2, nvec)); DFT over j1.  With b1 == m
// (single pass) the row is produced by SRC (generation / data load) instead.
template <typename CR, typename TOut, int SRC, int KT>
__global__ __launch_bounds__(256) void lat_pass2_kernel(const cx<CR>* __restrict__ Y,
                                                        cx<TOut>* __restrict__ X, int64_t vstride,
                                                        const void* __restrict__ y, int y_f32,
                                                        int m, int b1, double scale,
                                                        const uint32_t* __restrict__ gen,
                                                        const uint32_t* __restrict__ colshift,
                                                        const Params* __restrict__ P, int d) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n1 = 1 << b1;
  const int stride = lds_stride(b1);
  cx<CR>* a = reinterpret_cast<cx<CR>*>(smem);
  cx<CR>* tw = a + stride;
  const int v = blockIdx.y, f2 = blockIdx.x;
  fill_twiddles<CR>(tw, b1);
  const size_t row = (size_t)v * vstride + (size_t)f2 * n1;
  for (int j1 = threadIdx.x; j1 < n1; j1 += blockDim.x) {
    cx<CR> val;
    if (b1 < m) {
      val = Y[row + j1];
    } else if (SRC == SRC_GEN) {
      val = {lat_col_value<CR, KT>(gen, colshift + (size_t)v * d, d, (uint32_t)j1, m, P), (CR)0};
    } else {
      val = {(CR)load_data(y, y_f32, SRC, v, (uint32_t)j1, m), (CR)0};
    }
    a[lds_at(0, stride, j1)] = val;
  }
  lds_fft<CR>(a, 1, b1, stride, tw);
  for (int f1 = threadIdx.x; f1 < n1; f1 += blockDim.x) {
    const cx<CR> val = a[lds_at(0, stride, bitrev_bits(f1, b1))];
    X[row + f1] = {(TOut)(val.x * (CR)scale), (TOut)(val.y * (CR)scale)};
  }
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
enum { SINK_Z = LAT_SINK_Z, SINK_REDUCE = LAT_SINK_REDUCE, SINK_REAL = LAT_SINK_REAL };

// derivative accumulation for one element: wv = adjoint value, u[q] digits
template <typename R, int KT, int D>
__device__ inline void accum_derivs(R wv, const uint32_t* u, const R* eta, R gam, int d,
                                    const Params* __restrict__ P, R* acc_eta, R* acc_b, R& acc_c) {
  constexpr bool ADAPT = KT == KT_DSIA;
  R K[D], f[D];
  R Ka[ADAPT ? D : 1][4];
#pragma unroll
  for (int j = 0; j < D; j++) {
    if (j < d) {
      if constexpr (ADAPT) {
        dsi_khat_all<R>(u[j], Ka[j]);
        K[j] = RT<R>::bw(P, 0) * Ka[j][0] + RT<R>::bw(P, 1) * Ka[j][1] + RT<R>::bw(P, 2) * Ka[j][2] +
               RT<R>::bw(P, 3) * Ka[j][3];
      } else {
        K[j] = kval<R, KT>(u[j], P);
      }
      f[j] = fma(eta[j], K[j], (R)1);
    } else {
      K[j] = 0;
      f[j] = 1;
    }
  }
  R pre[D];
  R run = gam * wv;
#pragma unroll
  for (int j = 0; j < D; j++) {
    pre[j] = run;
    if (j < d) run *= f[j];
  }
  acc_c += run;
  R suf = 1;
#pragma unroll
  for (int j = D - 1; j >= 0; j--) {
    if (j < d) {
      const R ps = pre[j] * suf * eta[j];
      acc_eta[j] = fma(ps, K[j], acc_eta[j]);
      if constexpr (ADAPT) {
#pragma unroll
        for (int q = 0; q < 4; q++) acc_b[q] = fma(ps, Ka[j][q], acc_b[q]);
      }
      suf *= f[j];
    }
  }
}

template <typename R, int KT, int D>
__device__ inline void reduce_store(const R* acc_eta, const R* acc_b, R acc_c, int d, double* red,
                                    double* out) {
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
    v = (KT == KT_DSIA) ? block_sum((double)acc_b[q], red) : 0.0;
    if (threadIdx.x == 0) out[1 + d + q] = v;
  }
}

// Pass A' (one block per row f2): DFT over f1 of omega (or its conjugate),
// then SINK_Z: twiddle e^{-2 pi i j1 f2 / n}, store Z[f2][j1];
// single pass (b1 == m): SINK_REDUCE (derivative reduction of Re) or
// SINK_REAL (store Re * scale in natural order).
template <typename CR, typename TIn, int SINK, int KT, int D>
__global__ __launch_bounds__(256) void lat_adjA_kernel(
    const cx<TIn>* __restrict__ W, cx<CR>* __restrict__ Z, double* __restrict__ real_out,
    int64_t vstride, int m, int b1, int conj_in, double scale, const uint32_t* __restrict__ gen,
    const uint32_t* __restrict__ colshift, const Params* __restrict__ P, int d,
    double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  const int n1 = 1 << b1;
  const int stride = lds_stride(b1);
  cx<CR>* a = reinterpret_cast<cx<CR>*>(smem);
  cx<CR>* tw = a + stride;
  const int v = blockIdx.y, f2 = blockIdx.x;
  fill_twiddles<CR>(tw, b1);
  const size_t row = (size_t)v * vstride + (size_t)f2 * n1;
  for (int f1 = threadIdx.x; f1 < n1; f1 += blockDim.x) {
    const cx<TIn> w = W[row + f1];
    a[lds_at(0, stride, f1)] = {(CR)w.x, conj_in ? -(CR)w.y : (CR)w.y};
  }
  lds_fft<CR>(a, 1, b1, stride, tw);
  if (SINK == SINK_Z) {
    for (int j1 = threadIdx.x; j1 < n1; j1 += blockDim.x) {
      const cx<CR> val = a[lds_at(0, stride, bitrev_bits(j1, b1))];
      const cx<double> t = twiddle64((int64_t)j1 * f2, m);
      Z[row + j1] = cmul<CR>(val, {(CR)t.x, (CR)t.y});
    }
  } else if (SINK == SINK_REAL) {
    for (int j1 = threadIdx.x; j1 < n1; j1 += blockDim.x)
      real_out[(size_t)v * ((size_t)1 << m) + j1] =
          (double)a[lds_at(0, stride, bitrev_bits(j1, b1))].x * scale;
  } else {
    CR acc_eta[D], acc_b[4] = {0, 0, 0, 0}, acc_c = 0, eta[D];
#pragma unroll
    for (int j = 0; j < D; j++) {
      acc_eta[j] = 0;
      eta[j] = j < d ? RT<CR>::eta(P, j) : (CR)0;
    }
    const CR gam = RT<CR>::gamma(P);
    const uint32_t* sh = colshift + (size_t)v * d;
    for (int j1 = threadIdx.x; j1 < n1; j1 += blockDim.x) {
      uint32_t u[D];
#pragma unroll
      for (int q = 0; q < D; q++) u[q] = q < d ? lat_z(gen[q], (uint32_t)j1, m) + sh[q] : 0u;
      accum_derivs<CR, KT, D>(a[lds_at(0, stride, bitrev_bits(j1, b1))].x, u, eta, gam, d, P, acc_eta,
                              acc_b, acc_c);
    }
    reduce_store<CR, KT, D>(acc_eta, acc_b, acc_c, d, red,
                            partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * adj_nq(d));
  }
}

// Pass B' (tile = KC consecutive j1 x n2 rows f2; grid (n1 / KC, nvec)): DFT
// over f2 -> j2, then SINK_REDUCE or SINK_REAL on u(j1 + n1 j2) = Re.
template <typename CR, int SINK, int KT, int D>
__global__ __launch_bounds__(256) void lat_adjB_kernel(
    const cx<CR>* __restrict__ Z, double* __restrict__ real_out, int64_t vstride, int m, int b1,
    int KC, double scale, const uint32_t* __restrict__ gen, const uint32_t* __restrict__ colshift,
    const Params* __restrict__ P, int d, double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[16];
  const int b2 = m - b1, n1 = 1 << b1;
  const int stride = lds_stride(b2);
  cx<CR>* a = reinterpret_cast<cx<CR>*>(smem);
  cx<CR>* tw = a + (size_t)KC * stride;
  const int v = blockIdx.y;
  const int j1_0 = blockIdx.x * KC;
  fill_twiddles<CR>(tw, b2);
  const int kcb = __ffs(KC) - 1;
  const cx<CR>* zin = Z + (size_t)v * vstride;
  for (int q = threadIdx.x; q < (KC << b2); q += blockDim.x) {
    const int kc = q & (KC - 1), f2 = q >> kcb;
    a[lds_at(kc, stride, f2)] = zin[(size_t)f2 * n1 + j1_0 + kc];
  }
  lds_fft<CR>(a, KC, b2, stride, tw);
  if (SINK == SINK_REAL) {
    for (int q = threadIdx.x; q < (KC << b2); q += blockDim.x) {
      const int kc = q & (KC - 1), j2 = q >> kcb;
      const size_t j = (size_t)(j1_0 + kc) + ((size_t)j2 << b1);
      real_out[(size_t)v * ((size_t)1 << m) + j] =
          (double)a[lds_at(kc, stride, bitrev_bits(j2, b2))].x * scale;
    }
    return;
  }
  CR acc_eta[D], acc_b[4] = {0, 0, 0, 0}, acc_c = 0, eta[D];
#pragma unroll
  for (int j = 0; j < D; j++) {
    acc_eta[j] = 0;
    eta[j] = j < d ? RT<CR>::eta(P, j) : (CR)0;
  }
  const CR gam = RT<CR>::gamma(P);
  const uint32_t* sh = colshift + (size_t)v * d;
  for (int q = threadIdx.x; q < (KC << b2); q += blockDim.x) {
    const int kc = q & (KC - 1), j2 = q >> kcb;
    const uint32_t j = (uint32_t)(j1_0 + kc) + ((uint32_t)j2 << b1);
    uint32_t u[D];
#pragma unroll
    for (int qq = 0; qq < D; qq++) u[qq] = qq < d ? lat_z(gen[qq], j, m) + sh[qq] : 0u;
    accum_derivs<CR, KT, D>(a[lds_at(kc, stride, bitrev_bits(j2, b2))].x, u, eta, gam, d, P,
                            acc_eta, acc_b, acc_c);
  }
  reduce_store<CR, KT, D>(acc_eta, acc_b, acc_c, d, red,
                          partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * adj_nq(d));
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int lat_b1(int m) { return m < 12 ? m : 12; }
static int lat_kc(int m, int b1, size_t cbytes) {
  const int b2 = m - b1;
  int KC = 1;
  while (2 * KC <= (1 << b1) && (size_t)(2 * KC) * lds_stride(b2) * cbytes <= 32768) KC *= 2;
  return KC;
}
static size_t lds_pass1(int m, int b1, int KC, size_t cbytes) {
  const int b2 = m - b1;
  return ((size_t)KC * lds_stride(b2) + (b2 ? (1u << (b2 - 1)) : 0)) * cbytes;
}
static size_t lds_pass2(int b1, size_t cbytes) {
  return ((size_t)lds_stride(b1) + (b1 ? (1u << (b1 - 1)) : 0)) * cbytes;
}

int lat_adj_blocks(int m, size_t cbytes) {
  const int b1 = lat_b1(m);
  if (b1 == m) return 1;
  return (1 << b1) / lat_kc(m, b1, cbytes);
}

#define MTGP_LAT_KT(kt, MACRO, ...)                     \
  do {                                                  \
    switch (kt) {                                       \
      case KT_SI1: MACRO(KT_SI1, __VA_ARGS__); break;   \
      case KT_SI2: MACRO(KT_SI2, __VA_ARGS__); break;   \
      default: MACRO(KT_SI3, __VA_ARGS__); break;       \
    }                                                   \
  } while (0)

// Forward transform of nvec vectors (columns when src == SRC_GEN, data when
// SRC_Y) of length 2^m into the spectrum layout; `work` holds pass-1 output.
template <typename CR, typename SR>
int launch_lat_forward(int src, cx<CR>* work, cx<SR>* spec, int64_t vstride, int nvec, int m,
                       const void* y, int y_f32, double scale, const uint32_t* gen,
                       const uint32_t* colshift, const Params* P, const KDesc& kd,
                       hipStream_t st) {
  if (nvec <= 0) return 0;
  const int b1 = lat_b1(m);
  const int kt = kt_of(kd.family, kd.order, kd.adaptive);
  const size_t cb = sizeof(cx<CR>);
  if (b1 < m) {
    const int KC = lat_kc(m, b1, cb);
    const dim3 grid((1u << b1) / KC, nvec);
    const size_t lds = lds_pass1(m, b1, KC, cb);
#define P1(KTV, SRCV)                                                                              \
  hipLaunchKernelGGL((lat_pass1_kernel<CR, SRCV, KTV>), grid, dim3(256), lds, st, work, vstride, y, \
                     y_f32, m, b1, KC, gen, colshift, P, kd.d)
    if (src == SRC_GEN) MTGP_LAT_KT(kt, P1, SRC_GEN);
    else if (src == SRC_Y) P1(KT_SI1, SRC_Y);
    else P1(KT_SI1, SRC_X);
#undef P1
  }
  const dim3 grid2(1u << (m - b1), nvec);
  const size_t lds2 = lds_pass2(b1, cb);
#define P2(KTV, SRCV)                                                                           \
  hipLaunchKernelGGL((lat_pass2_kernel<CR, SR, SRCV, KTV>), grid2, dim3(256), lds2, st, work,   \
                     spec, vstride, y, y_f32, m, b1, scale, gen, colshift, P, kd.d)
  if (src == SRC_GEN) MTGP_LAT_KT(kt, P2, SRC_GEN);
  else if (src == SRC_Y) P2(KT_SI1, SRC_Y);
  else P2(KT_SI1, SRC_X);
#undef P2
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Adjoint: u = Re F omega, reduced against the regenerated column derivatives
// (partials: lat_adj_blocks(m) * nvec rows), or written (SINK_REAL, scaled) to
// real_out in natural order.
template <typename CR, typename SR>
int launch_lat_adjoint(int sink, const cx<SR>* spec, cx<CR>* work, double* real_out,
                       int64_t vstride, int nvec, int m, int conj_in, double scale,
                       const uint32_t* gen, const uint32_t* colshift, const Params* P,
                       const KDesc& kd, double* partials, hipStream_t st) {
  if (nvec <= 0) return 0;
  const int b1 = lat_b1(m);
  const int kt = kt_of(kd.family, kd.order, kd.adaptive);
  const size_t cb = sizeof(cx<CR>);
  const size_t ldsA = lds_pass2(b1, cb);
  const dim3 gridA(1u << (m - b1), nvec);
#define PA(DD, KTV, SINKV)                                                                        \
  hipLaunchKernelGGL((lat_adjA_kernel<CR, SR, SINKV, KTV, DD>), gridA, dim3(256), ldsA, st, spec,  \
                     work, real_out, vstride, m, b1, conj_in, scale, gen, colshift, P, kd.d,     \
                     partials)
  if (b1 < m) {
    PA(4, KT_SI1, SINK_Z);
    const int KC = lat_kc(m, b1, cb);
    const dim3 gridB((1u << b1) / KC, nvec);
    const size_t ldsB = lds_pass1(m, b1, KC, cb);
#define PB(DD, KTV, SINKV)                                                                        \
  hipLaunchKernelGGL((lat_adjB_kernel<CR, SINKV, KTV, DD>), gridB, dim3(256), ldsB, st, work,     \
                     real_out, vstride, m, b1, KC, scale, gen, colshift, P, kd.d, partials)
#define PB_KT(KTV, DD) PB(DD, KTV, SINK_REDUCE)
#define PB_D(DD, KTV) PB_KT(KTV, DD)
    if (sink == SINK_REAL) {
      PB(4, KT_SI1, SINK_REAL);
    } else {
      switch (kt) {
        case KT_SI1: MTGP_DISPATCH_D(kd.d, PB_D, KT_SI1); break;
        case KT_SI2: MTGP_DISPATCH_D(kd.d, PB_D, KT_SI2); break;
        default: MTGP_DISPATCH_D(kd.d, PB_D, KT_SI3); break;
      }
    }
#undef PB_D
#undef PB_KT
#undef PB
  } else {
#define PA_D(DD, KTV) PA(DD, KTV, SINK_REDUCE)
    if (sink == SINK_REAL) {
      PA(4, KT_SI1, SINK_REAL);
    } else {
      switch (kt) {
        case KT_SI1: MTGP_DISPATCH_D(kd.d, PA_D, KT_SI1); break;
        case KT_SI2: MTGP_DISPATCH_D(kd.d, PA_D, KT_SI2); break;
        default: MTGP_DISPATCH_D(kd.d, PA_D, KT_SI3); break;
      }
    }
#undef PA_D
  }
#undef PA
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_lat_forward<double, double>(int, cx<double>*, cx<double>*, int64_t, int, int,
                                                const void*, int, double, const uint32_t*,
                                                const uint32_t*, const Params*, const KDesc&,
                                                hipStream_t);
template int launch_lat_forward<double, float>(int, cx<double>*, cx<float>*, int64_t, int, int,
                                               const void*, int, double, const uint32_t*,
                                               const uint32_t*, const Params*, const KDesc&,
                                               hipStream_t);
template int launch_lat_forward<float, float>(int, cx<float>*, cx<float>*, int64_t, int, int,
                                              const void*, int, double, const uint32_t*,
                                              const uint32_t*, const Params*, const KDesc&,
                                              hipStream_t);

// spectrum layout (p = f2 n1 + f1 for f = f2 + n2 f1) -> natural frequency order
template <typename R>
__global__ void lat_natural_kernel(const cx<R>* __restrict__ spec, cx<R>* __restrict__ X,
                                   int64_t nvec, int m, int b1) {
  const int64_t n = (int64_t)1 << m;
  const int b2 = m - b1;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nvec * n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = q >> m, f = q & (n - 1);
    const int64_t f2 = f & ((1 << b2) - 1), f1 = f >> b2;
    X[q] = spec[v * n + (f2 << b1) + f1];
  }
}

int launch_lat_natural(const void* spec, int spec_f32, void* X, int64_t nvec, int m,
                       hipStream_t st) {
  const int64_t total = nvec << m;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  if (spec_f32)
    hipLaunchKernelGGL(lat_natural_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<const cx<float>*>(spec), static_cast<cx<float>*>(X), nvec, m,
                       lat_b1(m));
  else
    hipLaunchKernelGGL(lat_natural_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<const cx<double>*>(spec), static_cast<cx<double>*>(X), nvec, m,
                       lat_b1(m));
  return hipGetLastError() == hipSuccess ? 0 : -1;
}
template int launch_lat_adjoint<double, double>(int, const cx<double>*, cx<double>*, double*,
                                                int64_t, int, int, int, double, const uint32_t*,
                                                const uint32_t*, const Params*, const KDesc&,
                                                double*, hipStream_t);
template int launch_lat_adjoint<double, float>(int, const cx<float>*, cx<double>*, double*, int64_t,
                                               int, int, int, double, const uint32_t*,
                                               const uint32_t*, const Params*, const KDesc&,
                                               double*, hipStream_t);
template int launch_lat_adjoint<float, float>(int, const cx<float>*, cx<float>*, double*, int64_t,
                                              int, int, int, double, const uint32_t*,
                                              const uint32_t*, const Params*, const KDesc&, double*,
                                              hipStream_t);

}  // namespace mtgp

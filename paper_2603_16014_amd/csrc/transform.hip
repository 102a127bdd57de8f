// Transform passes over kernel columns and data vectors.
//
// A length-2^m Walsh-Hadamard transform (the V^dagger of Theorem "Fast GP
// computations" for digital sequences, unnormalised) is split by index bits:
//   pass A: bits [0, LB) of contiguous 2^LB blocks, LDS resident.  For kernel
//           columns the block is generated in registers first (fused column
//           evaluation, Eq. prod_kernel), so raw columns never reach HBM.
//   pass B: bits [lo, hi) (hi - lo <= 11), tiles of KC consecutive low indices
//           times 2^(hi-lo) strided rows, LDS resident.
// The stages of a Walsh-Hadamard transform commute, so the split needs no
// twiddles and the output stays in natural (Sylvester) order.
#include "kernels.h"

namespace mtgp {

// ---------------------------------------------------------------------------
// per-block table of uniform digit offsets: S[k][j] for element t + 256 k
//   DSEQ: z(i0 + 256 k) XOR shift_j  -> u = z(t) XOR S
//   LAT:  ((i0 + 256 k) g_j << (32 - m)) + shift_j  -> u = (t g_j << (32-m)) + S
// ---------------------------------------------------------------------------
template <int FAM>
__device__ inline void fill_offsets(uint32_t* S, int E, int d, uint32_t i0, int m,
                                    const uint32_t* __restrict__ gen,
                                    const uint32_t* __restrict__ sh) {
  for (int q = threadIdx.x; q < E * d; q += blockDim.x) {
    const int k = q / d, j = q - k * d;
    const uint32_t idx = i0 + 256u * (uint32_t)k;
    uint32_t v;
    if (FAM == FAM_DSEQ) {
      v = dseq_z(gen + 32 * j, idx) ^ sh[j];
    } else {
      v = lat_z(gen[j], idx, m) + sh[j];
    }
    S[k * d + j] = v;
  }
}

template <int FAM>
__device__ inline uint32_t thread_digit(const uint32_t* __restrict__ gen, int j, uint32_t t,
                                        int m) {
  if (FAM == FAM_DSEQ) return dseq_z(gen + 32 * j, t);
  return lat_z(gen[j], t, m);
}

template <int FAM>
__device__ inline uint32_t combine(uint32_t a, uint32_t s) {
  return FAM == FAM_DSEQ ? (a ^ s) : (a + s);
}

// Kernel column values for elements t + 256 k of the block starting at i0.
template <typename Real, int FAM, int ADAPT>
__device__ inline void column_values(Real* c, int E, int nb, uint32_t t, const uint32_t* S,
                                     const uint32_t* __restrict__ gen, int m,
                                     const Params* __restrict__ P, const KDesc& kd) {
  const Real g = RT<Real>::gamma(P);
#pragma unroll
  for (int k = 0; k < MAXE; k++) c[k] = g;
  for (int j = 0; j < kd.d; j++) {
    const uint32_t a = thread_digit<FAM>(gen, j, t, m);
    const Real eta = RT<Real>::eta(P, j);
#pragma unroll
    for (int k = 0; k < MAXE; k++) {
      if (k < E && (int)t + 256 * k < nb) {
        const uint32_t u = combine<FAM>(a, S[k * kd.d + j]);
        c[k] *= (Real)1 + eta * univ_value<Real, FAM, ADAPT>(kd.order, u, P);
      }
    }
  }
}

// Pass A with fused column generation: grid (2^(m-LB), ncols).  Arithmetic in
// Real; the block is stored as TOut (the spectrum precision when this pass
// completes the transform, else the working precision).
template <typename Real, typename TOut, int FAM, int ADAPT, bool DO_FWHT>
__global__ __launch_bounds__(256) void gen_cols_kernel(TOut* __restrict__ base, int64_t col_stride,
                                                       int m, int LB,
                                                       const uint32_t* __restrict__ gen,
                                                       const uint32_t* __restrict__ colshift,
                                                       const Params* __restrict__ P, KDesc kd) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nb = 1 << LB;
  const int E = nb > 256 ? nb / 256 : 1;
  uint32_t* S = reinterpret_cast<uint32_t*>(smem);
  Real* lds = reinterpret_cast<Real*>(smem + sizeof(uint32_t) * MAXE * MTGP_MAXD);
  const int col = blockIdx.y;
  const uint32_t i0 = (uint32_t)blockIdx.x << LB;
  const uint32_t t = threadIdx.x;
  fill_offsets<FAM>(S, E, kd.d, i0, m, gen, colshift + (size_t)col * kd.d);
  __syncthreads();
  Real c[MAXE];
  column_values<Real, FAM, ADAPT>(c, E, nb, t, S, gen, m, P, kd);
  TOut* out = base + (size_t)col * col_stride + i0;
  if (!DO_FWHT) {
#pragma unroll
    for (int k = 0; k < MAXE; k++)
      if (k < E && (int)t + 256 * k < nb) out[t + 256 * k] = (TOut)c[k];
    return;
  }
  const int stride = lds_stride(LB);
#pragma unroll
  for (int k = 0; k < MAXE; k++)
    if (k < E && (int)t + 256 * k < nb) lds[lds_at(0, stride, t + 256 * k)] = c[k];
  lds_fwht<Real>(lds, 1, LB, stride);
#pragma unroll
  for (int k = 0; k < MAXE; k++)
    if (k < E && (int)t + 256 * k < nb) out[t + 256 * k] = (TOut)lds[lds_at(0, stride, t + 256 * k)];
}

// Pass A on data already in memory: grid (2^(m-LB), nvec); in place.
template <typename Real>
__global__ __launch_bounds__(256) void fwht_lo_kernel(Real* __restrict__ base, int64_t vec_stride,
                                                      int LB) {
  extern __shared__ __align__(16) unsigned char smem[];
  Real* lds = reinterpret_cast<Real*>(smem);
  const int nb = 1 << LB;
  const int stride = lds_stride(LB);
  Real* p = base + (size_t)blockIdx.y * vec_stride + ((size_t)blockIdx.x << LB);
  for (int i = threadIdx.x; i < nb; i += blockDim.x) lds[lds_at(0, stride, i)] = p[i];
  lds_fwht<Real>(lds, 1, LB, stride);
  for (int i = threadIdx.x; i < nb; i += blockDim.x) p[i] = lds[lds_at(0, stride, i)];
}

// Pass B: butterflies over bits [lo, lo + hb) of vectors of length 2^m.
// Tile = KC consecutive low indices x 2^hb rows; grid (2^lo / KC * 2^(m-lo-hb), nvec).
// Arithmetic in TIn; the result is stored as TOut (in place when in == out).
template <typename TIn, typename TOut>
__global__ __launch_bounds__(256) void fwht_strided_kernel(const TIn* in, TOut* out,
                                                           int64_t vec_stride, int m, int lo,
                                                           int hb, int KC) {
  extern __shared__ __align__(16) unsigned char smem[];
  TIn* lds = reinterpret_cast<TIn*>(smem);
  const int tiles_lo = (1 << lo) / KC;
  const int tl = blockIdx.x % tiles_lo;
  const int ch = blockIdx.x / tiles_lo;
  const int hi = lo + hb;
  const size_t off = (size_t)blockIdx.y * vec_stride + (size_t)tl * KC + ((size_t)ch << hi);
  const TIn* p = in + off;
  TOut* q_out = out + off;
  const int rows = 1 << hb;
  const int stride = lds_stride(hb);
  const int total = rows * KC;
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int kc = q % KC, r = q / KC;
    lds[lds_at(kc, stride, r)] = p[kc + ((size_t)r << lo)];
  }
  lds_fwht<TIn>(lds, KC, hb, stride);
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int kc = q % KC, r = q / KC;
    q_out[kc + ((size_t)r << lo)] = (TOut)lds[lds_at(kc, stride, r)];
  }
}

template <typename Real>
__global__ void scale_kernel(Real* __restrict__ x, int64_t n, Real s) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] *= s;
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
size_t gen_cols_lds_bytes(int LB, int real_bytes) {
  return sizeof(uint32_t) * MAXE * MTGP_MAXD + (size_t)lds_stride(LB) * real_bytes;
}

// All passes over bits [lb(m), m): arithmetic in TIn on `work` in place; the
// last pass writes `out` as TOut (which may alias `work` when TIn == TOut).
template <typename TIn, typename TOut>
static int launch_strided_passes(TIn* work, TOut* out, int64_t vec_stride, int64_t nvec, int m,
                                 const Sched& sc, hipStream_t st) {
  int lo = sc.lb(m);
  while (lo < m) {
    const int hb = (m - lo) < sc.b_bits ? (m - lo) : sc.b_bits;
    const bool last = lo + hb >= m;
    // largest power of two KC with KC padded sequences inside the tile budget
    int KC = 1;
    while ((size_t)(2 * KC) * lds_stride(hb) * sizeof(TIn) <= sc.b_tile && 2 * KC <= (1 << lo))
      KC *= 2;
    const int64_t tiles = ((int64_t)1 << lo) / KC * ((int64_t)1 << (m - lo - hb));
    const size_t lds = (size_t)KC * lds_stride(hb) * sizeof(TIn);
    for (int64_t v0 = 0; v0 < nvec; v0 += 65535) {
      const int64_t nv = (nvec - v0) < 65535 ? (nvec - v0) : 65535;
      if (last)
        hipLaunchKernelGGL((fwht_strided_kernel<TIn, TOut>), dim3((unsigned)tiles, (unsigned)nv),
                           dim3(256), lds, st, work + v0 * vec_stride, out + v0 * vec_stride,
                           vec_stride, m, lo, hb, KC);
      else
        hipLaunchKernelGGL((fwht_strided_kernel<TIn, TIn>), dim3((unsigned)tiles, (unsigned)nv),
                           dim3(256), lds, st, work + v0 * vec_stride, work + v0 * vec_stride,
                           vec_stride, m, lo, hb, KC);
    }
    lo += hb;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename Real>
int launch_fwht(Real* base, int64_t vec_stride, int64_t nvec, int m, const Sched& sc,
                hipStream_t st) {
  if (nvec <= 0) return 0;
  const int LB = sc.lb(m);
  const size_t lds = (size_t)lds_stride(LB) * sizeof(Real);
  for (int64_t v0 = 0; v0 < nvec; v0 += 65535) {
    const int64_t nv = (nvec - v0) < 65535 ? (nvec - v0) : 65535;
    hipLaunchKernelGGL(fwht_lo_kernel<Real>, dim3(1u << (m - LB), (unsigned)nv), dim3(256), lds, st,
                       base + v0 * vec_stride, vec_stride, LB);
  }
  return launch_strided_passes<Real, Real>(base, base, vec_stride, nvec, m, sc, st);
}

template <typename TIn, typename TOut>
int launch_fwht_high(TIn* work, TOut* out, int64_t vec_stride, int64_t nvec, int m,
                     const Sched& sc, hipStream_t st) {
  return launch_strided_passes<TIn, TOut>(work, out, vec_stride, nvec, m, sc, st);
}

template <typename Real, typename TOut>
int launch_gen_cols(TOut* base, int64_t col_stride, int ncols, int m, const uint32_t* gen,
                    const uint32_t* colshift, const Params* P, const KDesc& kd, bool do_fwht,
                    const Sched& sc, hipStream_t st) {
  if (ncols <= 0) return 0;
  const int LB = sc.lb(m);
  const size_t lds = gen_cols_lds_bytes(LB, sizeof(Real));
  dim3 grid(1u << (m - LB), (unsigned)ncols);
#define MTGP_GEN(F, A, W)                                                                      \
  hipLaunchKernelGGL((gen_cols_kernel<Real, TOut, F, A, W>), grid, dim3(256), lds, st, base,   \
                     col_stride, m, LB, gen, colshift, P, kd)
  if (kd.family == FAM_DSEQ) {
    if (kd.adaptive) {
      if (do_fwht) MTGP_GEN(FAM_DSEQ, 1, true); else MTGP_GEN(FAM_DSEQ, 1, false);
    } else {
      if (do_fwht) MTGP_GEN(FAM_DSEQ, 0, true); else MTGP_GEN(FAM_DSEQ, 0, false);
    }
  } else {
    if (do_fwht) MTGP_GEN(FAM_LAT, 0, true); else MTGP_GEN(FAM_LAT, 0, false);
  }
#undef MTGP_GEN
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <typename Real>
int launch_scale(Real* x, int64_t n, Real s, hipStream_t st) {
  if (n <= 0) return 0;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(scale_kernel<Real>, dim3((unsigned)blocks), dim3(256), 0, st, x, n, s);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_fwht<double>(double*, int64_t, int64_t, int, const Sched&, hipStream_t);
template int launch_fwht<float>(float*, int64_t, int64_t, int, const Sched&, hipStream_t);
template int launch_fwht_high<double, double>(double*, double*, int64_t, int64_t, int,
                                              const Sched&, hipStream_t);
template int launch_fwht_high<double, float>(double*, float*, int64_t, int64_t, int, const Sched&,
                                             hipStream_t);
template int launch_fwht_high<float, float>(float*, float*, int64_t, int64_t, int, const Sched&,
                                            hipStream_t);
template int launch_gen_cols<double, double>(double*, int64_t, int, int, const uint32_t*,
                                             const uint32_t*, const Params*, const KDesc&, bool,
                                             const Sched&, hipStream_t);
template int launch_gen_cols<double, float>(float*, int64_t, int, int, const uint32_t*,
                                            const uint32_t*, const Params*, const KDesc&, bool,
                                            const Sched&, hipStream_t);
template int launch_gen_cols<float, float>(float*, int64_t, int, int, const uint32_t*,
                                           const uint32_t*, const Params*, const KDesc&, bool,
                                           const Sched&, hipStream_t);
template int launch_scale<double>(double*, int64_t, double, hipStream_t);
template int launch_scale<float>(float*, int64_t, float, hipStream_t);

}  // namespace mtgp

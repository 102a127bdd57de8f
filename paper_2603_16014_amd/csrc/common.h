// Device-side building blocks shared by the HIP kernels of the fast MTGP
// library (gfx950, wave64).
//
//  * Params: the decoded hyperparameters (written by the prep kernel from the
//    packed theta vector), read by every other kernel.
//  * Univariate kernels on 32-bit digits: adaptive-smoothness DSI kernels
//    Khat_1..Khat_4 (Eq. DSI_kernel_1d_ex; Khat_1 read as 1 - 3 t_1, the
//    zero-mean order-one Walsh kernel) and SI Bernoulli kernels (Eq.
//    SI_kernel_1d_ex).
//  * Point generation helpers: digital sequences (XOR of generating columns
//    over the set bits of the index, Def. "Base-2 digitally-shifted digital
//    sequences") and rank-1 lattices in natural order (j g / n mod 1).
//  * LDS Walsh-Hadamard rounds: radix-2^r butterflies over a group of index
//    bits, used by every transform pass.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MTGP_MAXT 16
#define MTGP_MAXD 32
#define MTGP_MAXS 16

namespace mtgp {

enum Family { FAM_DSEQ = 0, FAM_LAT = 1 };

// Decoded hyperparameters; one copy lives at the start of the workspace.
struct Params {
  double gamma;
  double eta[MTGP_MAXD];
  double b[4];
  double xi[MTGP_MAXT];
  double zeta[MTGP_MAXT];
  double tau[MTGP_MAXT];
  double tau_used[MTGP_MAXT];  // means of the last loss evaluation (tau_hat or tau)
  double R[MTGP_MAXT * MTGP_MAXT];
  double B[MTGP_MAXT * MTGP_MAXS];
  // Pi = E Ktilde^-1 E^T of the last unequal-size loss (row-major, MAXT wide)
  double Pi[MTGP_MAXT * MTGP_MAXT];
  // q = r^T Ktilde^-2 r and s = tr Ktilde^-1 of the last GCV loss
  double gcv_q, gcv_s;
  float gamma_f;
  float eta_f[MTGP_MAXD];
  float b_f[4];
};

// Static description of a plan that kernels need, passed by value.
struct KDesc {
  int T, d, family, order, adaptive, s, profile;
  int unequal;        // nested unequal sizes (Algorithm 1 path)
  int gcv;            // the solves computed the GCV loss (q, s) instead of the MLE loss
  int m[MTGP_MAXT];   // per-task log2 sizes
};

// ---------------------------------------------------------------------------
// precision traits
// ---------------------------------------------------------------------------
template <typename Real> struct RT;
template <> struct RT<double> {
  __device__ static inline double unit(uint32_t u) { return (double)u * 0x1p-32; }
  // 2^-e for 0 <= e < 1023, built from the exponent field
  __device__ static inline double pow2neg(int e) { return __hiloint2double((1023 - e) << 20, 0); }
  __device__ static inline double gamma(const Params* p) { return p->gamma; }
  __device__ static inline double eta(const Params* p, int j) { return p->eta[j]; }
  __device__ static inline double bw(const Params* p, int a) { return p->b[a]; }
};
template <> struct RT<float> {
  // x = u 2^-32 rounded to float; a value that rounds to 1 is mapped to the
  // largest float below 1 (the boundary convention for points equal to 1)
  __device__ static inline float unit(uint32_t u) {
    return fminf((float)u * 0x1p-32f, 0x1.fffffep-1f);
  }
  __device__ static inline float pow2neg(int e) { return __int_as_float((127 - e) << 23); }
  __device__ static inline float gamma(const Params* p) { return p->gamma_f; }
  __device__ static inline float eta(const Params* p, int j) { return p->eta_f[j]; }
  __device__ static inline float bw(const Params* p, int a) { return p->b_f[a]; }
};

// ---------------------------------------------------------------------------
// univariate kernels on digits
// ---------------------------------------------------------------------------
// sum_{a=1..32} x_a 8^-(a-1) for x = u 2^-32 with binary digits x_a
__device__ inline uint64_t spread3_21(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}
__device__ inline double octal_digit_sum(uint32_t u) {
  // digits 1..21 (top 21 bits) then digits 22..32 (low 11 bits)
  uint64_t hi = spread3_21(u >> 11);
  uint64_t lo = spread3_21(u & 0x7ffu);
  return (double)hi * 0x1p-60 + (double)lo * 0x1p-93;
}

// beta(x) = -floor(log2 x) with beta(0) = 0, and t_1(x) = 2^-beta(x) with
// t_1(0) = 0.  t_1 is the leading power of two of x: x with its mantissa bits
// cleared (x = 0 stays 0).  In FP32 the digit is converted by truncation so
// that x never rounds up across a power of two (consistent with beta).
template <typename Real> __device__ inline Real lead_pow2(Real x);
template <> __device__ inline double lead_pow2<double>(double x) {
  return __hiloint2double(__double2hiint(x) & 0x7ff00000, 0);
}
template <> __device__ inline float lead_pow2<float>(float x) {
  return __int_as_float(__float_as_int(x) & 0x7f800000);
}
template <typename Real> __device__ inline Real unit_trunc(uint32_t u);
template <> __device__ inline double unit_trunc<double>(uint32_t u) { return (double)u * 0x1p-32; }
template <> __device__ inline float unit_trunc<float>(uint32_t u) { return __uint2float_rz(u) * 0x1p-32f; }

// beta(u) = (index of the leading 1 digit) = clz(u) + 1, beta(0) = 0.  The
// find-first-bit-high instruction returns -1 for u = 0, so adding 1 gives
// both cases without a compare and select.
__device__ inline int beta_of(uint32_t u) {
  int r;
  asm("v_ffbh_u32 %0, %1" : "=v"(r) : "v"(u));
  return r + 1;
}

// Khat_alpha(x), x = u 2^-32 (Eq. DSI_kernel_1d_ex), beta(0) = t_nu(0) = 0.
template <typename Real, int ORDER>
__device__ inline Real dsi_khat_o(uint32_t u) {
  const Real x = unit_trunc<Real>(u);
  const Real t1 = lead_pow2<Real>(x);
  if (ORDER == 1) return fma((Real)-3, t1, (Real)1);
  const Real b = (Real)beta_of(u);
  if (ORDER == 2) return fma(-b, x, fma((Real)-2.5, t1, (Real)1.5));
  const Real t2 = t1 * t1;
  if (ORDER == 3)
    return (Real)-1 + b * x * x - (Real)5 * ((Real)1 - t1) * x + (Real)(43.0 / 18.0) * ((Real)1 - t2);
  const Real t3 = t2 * t1;
  const Real s = (Real)(8.0 / 7.0) - (Real)2 * (Real)octal_digit_sum(u);
  return (Real)-1 - (Real)(2.0 / 3.0) * b * x * x * x + (Real)5 * ((Real)1 - t1) * x * x -
         (Real)(43.0 / 9.0) * ((Real)1 - t2) * x + (Real)(701.0 / 294.0) * ((Real)1 - t3) +
         b * (s * (Real)(1.0 / 48.0) - (Real)(1.0 / 42.0));
}

template <typename Real>
__device__ inline Real dsi_khat(int order, uint32_t u) {
  switch (order) {
    case 1: return dsi_khat_o<Real, 1>(u);
    case 2: return dsi_khat_o<Real, 2>(u);
    case 3: return dsi_khat_o<Real, 3>(u);
    default: return dsi_khat_o<Real, 4>(u);
  }
}

// all four Khat_alpha at once (adaptive kernel), sharing beta, x, t_nu
template <typename Real>
__device__ inline void dsi_khat_all(uint32_t u, Real k[4]) {
  const Real x = unit_trunc<Real>(u);
  const Real b = (Real)beta_of(u);
  const Real t1 = lead_pow2<Real>(x), t2 = t1 * t1, t3 = t2 * t1;
  const Real s = (Real)(8.0 / 7.0) - (Real)2 * (Real)octal_digit_sum(u);
  k[0] = fma((Real)-3, t1, (Real)1);
  k[1] = fma(-b, x, fma((Real)-2.5, t1, (Real)1.5));
  k[2] = (Real)-1 + b * x * x - (Real)5 * ((Real)1 - t1) * x + (Real)(43.0 / 18.0) * ((Real)1 - t2);
  k[3] = (Real)-1 - (Real)(2.0 / 3.0) * b * x * x * x + (Real)5 * ((Real)1 - t1) * x * x -
         (Real)(43.0 / 9.0) * ((Real)1 - t2) * x + (Real)(701.0 / 294.0) * ((Real)1 - t3) +
         b * (s * (Real)(1.0 / 48.0) - (Real)(1.0 / 42.0));
}

// (-1)^(alpha+1) (2 pi)^(2 alpha) / (2 alpha)! B_{2 alpha}(x) (Eq. SI_kernel_1d_ex)
template <typename Real>
__device__ inline Real si_kern(int order, uint32_t u) {
  const Real x = RT<Real>::unit(u);
  const Real x2 = x * x;
  switch (order) {
    case 1:  // 2 pi^2 (x^2 - x + 1/6)
      return (Real)19.739208802178716 * (x2 - x + (Real)(1.0 / 6.0));
    case 2:  // -(2/3) pi^4 (x^4 - 2x^3 + x^2 - 1/30)
      return (Real)-64.939394022668291 * (x2 * (x2 - (Real)2 * x + (Real)1) - (Real)(1.0 / 30.0));
    default:  // (4/45) pi^6 (x^6 - 3x^5 + 5/2 x^4 - 1/2 x^2 + 1/42)
      return (Real)85.456817206693727 *
             (x2 * (x2 * (x2 - (Real)3 * x + (Real)2.5) - (Real)0.5) + (Real)(1.0 / 42.0));
  }
}

// univariate kernel value for a (non-adaptive) family/order
template <typename Real, int FAM>
__device__ inline Real univ(int order, uint32_t u) {
  if (FAM == FAM_DSEQ) return dsi_khat<Real>(order, u);
  return si_kern<Real>(order, u);
}

// Kernel types known at compile time: DSI orders 1..4, the adaptive DSI
// kernel, SI orders 1..3.
enum KType { KT_DSI1 = 1, KT_DSI2 = 2, KT_DSI3 = 3, KT_DSI4 = 4, KT_DSIA = 5,
             KT_SI1 = 11, KT_SI2 = 12, KT_SI3 = 13 };
__host__ __device__ constexpr int kt_family(int kt) { return kt >= 11 ? FAM_LAT : FAM_DSEQ; }
__host__ inline int kt_of(int family, int order, int adaptive) {
  if (family == FAM_LAT) return 10 + order;
  return adaptive ? KT_DSIA : order;
}

// ---------------------------------------------------------------------------
// points
// ---------------------------------------------------------------------------
// z(i) of dimension j for a digital sequence: XOR of generating columns over
// the set bits of i (gen laid out [d][32]).
__device__ inline uint32_t dseq_z(const uint32_t* gen_j, uint32_t i) {
  uint32_t z = 0;
  while (i) {
    const int p = __ffs(i) - 1;
    z ^= gen_j[p];
    i &= i - 1;
  }
  return z;
}

// ---------------------------------------------------------------------------
// LDS Walsh-Hadamard rounds
// ---------------------------------------------------------------------------
// Sequences of length 2^L live in LDS at seq * stride + i + (i >> 4); the
// extra element per 16 (and a stride that is not a multiple of 32) keeps
// strided accesses off a single bank.
__host__ __device__ inline int lds_stride(int L) { return (1 << L) + ((1 << L) >> 4) + 1; }
__device__ inline int lds_at(int seq, int stride, int i) { return seq * stride + i + (i >> 4); }

// Butterflies over bits [lo, lo + R) of every one of nseq sequences.
template <typename Real, int R>
__device__ inline void lds_round(Real* lds, int nseq, int L, int lo, int stride) {
  const int ps_bits = L - R;  // groups per sequence = 2^ps_bits
  const int total = nseq << ps_bits;
  const int lo_mask = (1 << lo) - 1;
  const int q_mask = (1 << ps_bits) - 1;
  for (int g = threadIdx.x; g < total; g += blockDim.x) {
    const int seq = g >> ps_bits;
    const int q = g & q_mask;
    const int base = (q & lo_mask) | ((q >> lo) << (lo + R));
    Real v[1 << R];
#pragma unroll
    for (int k = 0; k < (1 << R); k++) v[k] = lds[lds_at(seq, stride, base + (k << lo))];
#pragma unroll
    for (int h = 1; h < (1 << R); h <<= 1) {
#pragma unroll
      for (int k = 0; k < (1 << R); k++) {
        if (!(k & h)) {
          const Real a = v[k], c = v[k + h];
          v[k] = a + c;
          v[k + h] = a - c;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < (1 << R); k++) lds[lds_at(seq, stride, base + (k << lo))] = v[k];
  }
}

// Full transform over bits [0, L) of nseq LDS sequences, in rounds of <= 4 bits.
template <typename Real>
__device__ inline void lds_fwht(Real* lds, int nseq, int L, int stride) {
  int lo = 0;
  while (lo < L) {
    const int r = min(4, L - lo);
    __syncthreads();
    switch (r) {
      case 4: lds_round<Real, 4>(lds, nseq, L, lo, stride); break;
      case 3: lds_round<Real, 3>(lds, nseq, L, lo, stride); break;
      case 2: lds_round<Real, 2>(lds, nseq, L, lo, stride); break;
      default: lds_round<Real, 1>(lds, nseq, L, lo, stride); break;
    }
    lo += r;
  }
  __syncthreads();
}

// Records a non-positive or non-finite pivot: status[0] |= 1 and the smallest
// offending index in the 64-bit word at status + 2.
__device__ inline void flag_bad(int* status, int64_t idx) {
  atomicOr(status, 1);
  atomicMin(reinterpret_cast<unsigned long long*>(status + 2), (unsigned long long)idx);
}

// ---------------------------------------------------------------------------
// raw buffer access
// ---------------------------------------------------------------------------
// A resource covers one window (at most 2^31 bytes) from a base address; an
// access takes the lane's byte offset in a vector register and a wave-uniform
// byte offset as a scalar, so strided rows cost one scalar each instead of a
// 64-bit vector address each.  Accesses outside the window read 0 and drop
// the store.
constexpr int kBufDword3 = 0x00020000;  // gfx9-family raw buffer format word
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, kBufDword3);
}

template <typename T>
__device__ inline T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 16)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  else if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

template <typename T>
__device__ inline void buf_store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 16)
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, voff, soff, 0);
  else if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}

// ---------------------------------------------------------------------------
// block reductions (FP64)
// ---------------------------------------------------------------------------
// Value of another lane of the row under a DPP control (rows whose bit in
// ROW_MASK is clear read 0).
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_read(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, true);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave, returned in every lane; every lane must be
// active.  DPP row operations (no LDS traffic): quad permutes and row mirrors
// give each lane its 16-lane row sum, two row broadcasts carry rows 0-2 into
// lane 63, which is read back through a scalar register.
__device__ inline double wave_sum(double v) {
  v += dpp_read<0xb1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_read<0x4e, 0xf>(v);   // quad_perm [2, 3, 0, 1]
  v += dpp_read<0x141, 0xf>(v);  // row_half_mirror: sums of 8
  v += dpp_read<0x140, 0xf>(v);  // row_mirror: sums of 16
  v += dpp_read<0x142, 0xa>(v);  // row_bcast15 into rows 1 and 3
  v += dpp_read<0x143, 0xc>(v);  // row_bcast31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// Sums v over the block; every thread gets the result.  `red` holds >= 16 doubles.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; i++) s += red[i];
  return s;
}

// Block reduction of NQ values per thread (q < nq used).  One barrier:
// each wave reduces in registers, lane 0 stores to red[wave][NQ], and the
// first nq threads add the per-wave rows in a fixed order (deterministic).
// `red` holds (blockDim.x / 64) * NQ doubles.
template <int NQ>
__device__ inline void block_sum_store(const double* vals, int nq, double* red, double* out) {
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int q = 0; q < NQ; q++) {
    if (q < nq) {
      const double v = wave_sum(vals[q]);
      if ((threadIdx.x & 63) == 0) red[w * NQ + q] = v;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < nw; i++) s += red[i * NQ + q];
    out[q] = s;
  }
}

// As block_sum_store over the first nred slots; the slots [nred, NQ) are
// nonzero only in thread 0 of block 0 (the thread of frequency 0), so each
// block's thread 0 stores its own values there instead of a block sum.
template <int NQ>
__device__ inline void block_sum_store_head(const double* vals, int nred, double* red,
                                            double* out) {
  block_sum_store<NQ>(vals, nred, red, out);
  if (threadIdx.x == 0)
    for (int q = nred; q < NQ; q++) out[q] = vals[q];
}

}  // namespace mtgp

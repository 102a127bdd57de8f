// Per-thread generation of kernel-column arguments inside a transform block.
//
// A block covers indices i0 + e, e < 2^LB; thread t owns e = t + 256 kk for
// kk = 0 .. E-1.  The digit of index i0 + t + 256 kk in dimension j splits
// into a per-thread part a_j (index t) and a part s_j that is the same for
// the whole block (indices i0 + 256 kk, plus the pair shift):
//   digital sequences: z(i) is XOR-linear in the bits of i, so
//     u_j = z_j(t) XOR z_j(i0 + 256 kk) XOR shift_j, and visiting kk in
//     Gray-code order changes s_j by one generating column per element
//     (the recursive identity x_{2^p + i} = x_{2^p} XOR x_i of Section
//     "Algorithm for Gram Matrix Calculations");
//   lattices (natural order j g / n): u_j = t g 2^(32-m) + (i0 + 256 kk) g
//     2^(32-m) + shift_j mod 2^32, advanced by one constant per element.
#pragma once
#include "kernels.h"

namespace mtgp {

template <int FAM, int D>
struct Digits {
  uint32_t a[D];     // per-thread part
  uint32_t s[D];     // block part of the current element (uniform)
  uint32_t step[D];  // lattice increment per element (uniform)

  // t < 256 (the nets' per-thread part XORs the generating columns 0 .. 7
  // selected by t's bits through masks: no per-lane chain of loads)
  __device__ inline void init(const uint32_t* __restrict__ gen, const uint32_t* __restrict__ sh,
                              int d, uint32_t t, uint32_t i0, int m) {
    uint32_t msk[8];
#pragma unroll
    for (int p = 0; p < 8; p++) msk[p] = 0u - ((t >> p) & 1u);
    // every slot is computed from a valid dimension (padding slots reuse
    // dimension 0) and masked afterwards, so no slot is indexed at run time
#pragma unroll
    for (int j = 0; j < D; j++) {
      const int jj = j < d ? j : 0;
      const uint32_t keep = j < d ? 0xffffffffu : 0u;
      if (FAM == FAM_DSEQ) {
        uint32_t z = 0;
#pragma unroll
        for (int p = 0; p < 8; p++) z ^= gen[32 * jj + p] & msk[p];
        a[j] = z & keep;
        s[j] = (dseq_z(gen + 32 * jj, i0) ^ sh[jj]) & keep;
        step[j] = 0;
      } else {
        a[j] = lat_z(gen[jj], t, m) & keep;
        s[j] = (lat_z(gen[jj], i0, m) + sh[jj]) & keep;
        step[j] = lat_z(gen[jj], 256u, m) & keep;
      }
    }
  }
  // block part only, for a new block start i0 (per-thread part unchanged)
  __device__ inline void set_block(const uint32_t* __restrict__ gen,
                                   const uint32_t* __restrict__ sh, int d, uint32_t i0, int m) {
#pragma unroll
    for (int j = 0; j < D; j++) {
      const int jj = j < d ? j : 0;
      const uint32_t keep = j < d ? 0xffffffffu : 0u;
      if (FAM == FAM_DSEQ) s[j] = (dseq_z(gen + 32 * jj, i0) ^ sh[jj]) & keep;
      else s[j] = (lat_z(gen[jj], i0, m) + sh[jj]) & keep;
    }
  }
  __device__ inline uint32_t u(int j) const { return FAM == FAM_DSEQ ? (a[j] ^ s[j]) : (a[j] + s[j]); }
  // element offset (in units of 256) visited at step k
  __device__ static inline int elem(int k) { return FAM == FAM_DSEQ ? (k ^ (k >> 1)) : k; }
  // move from step k to step k + 1 (padding slots XOR a masked column of
  // dimension 0, so the update is branch-free and stays in bounds)
  __device__ inline void advance(const uint32_t* __restrict__ gen, int d, int k) {
    if (FAM == FAM_DSEQ) {
      const int p = 8 + __ffs(k + 1) - 1;
#pragma unroll
      for (int j = 0; j < D; j++) {
        const int jj = j < d ? j : 0;
        const uint32_t keep = j < d ? 0xffffffffu : 0u;
        s[j] ^= gen[32 * jj + p] & keep;
      }
    } else {
#pragma unroll
      for (int j = 0; j < D; j++) s[j] += step[j];
    }
  }
};

// Digital-sequence digits for the fused kernels, with the block part folded
// into the per-thread part and the element part read from a table:
//   u_j(i0 + t + 256 gray(k)) = [z_j(t) ^ z_j(i0) ^ shift_j] ^ z_j(256 gray(k)),
// where gray(k) = k ^ (k >> 1) is the element visited at step k.  Row k of
// the table (GRAY_STRIDE words, 0 beyond the d dimensions) holds
// z_j(256 gray(k)); it depends on the generating matrices only, so one table
// serves every block and column, and a step costs one XOR per dimension with
// a wave-uniform (scalar) operand.  The table follows the d x 32 generating
// columns in the same buffer (gray_table).

template <int D>
struct FoldedDigits {
  uint32_t a[D];   // per-thread part with the block part folded in
  uint32_t s[D];   // element part z_j(256 gray(k)) of the current step (uniform)
  uint32_t nx[D];  // element part of the next step, read one step ahead (uniform)

  // t < 256.  z is XOR-linear, so z_j(t ^ i0) = z_j(t) ^ z_j(i0): the block
  // part z_j(i0) is wave-uniform, and the per-thread part XORs the generating
  // columns 0 .. 7 selected by t's bits through masks (no per-lane load chain).
  __device__ inline void init(const uint32_t* __restrict__ gen, const uint32_t* __restrict__ sh,
                              int d, uint32_t t, uint32_t i0) {
    uint32_t msk[8];
#pragma unroll
    for (int p = 0; p < 8; p++) msk[p] = 0u - ((t >> p) & 1u);
#pragma unroll
    for (int j = 0; j < D; j++) {
      const int jj = j < d ? j : 0;
      const uint32_t keep = j < d ? 0xffffffffu : 0u;
      const uint32_t* gj = gen + 32 * jj;
      uint32_t z = dseq_z(gj, i0) ^ sh[jj];
#pragma unroll
      for (int p = 0; p < 8; p++) z ^= gj[p] & msk[p];
      a[j] = z & keep;
      s[j] = 0;
    }
  }
  // from block start i0_old to i0 (the shift cancels: z is XOR-linear)
  __device__ inline void set_block(const uint32_t* __restrict__ gen, int d, uint32_t i0_old,
                                   uint32_t i0) {
#pragma unroll
    for (int j = 0; j < D; j++) {
      const int jj = j < d ? j : 0;
      const uint32_t keep = j < d ? 0xffffffffu : 0u;
      a[j] ^= dseq_z(gen + 32 * jj, i0_old ^ i0) & keep;
      s[j] = 0;
    }
  }
  // element part of step k (row 0 is zero)
  __device__ inline void load(const uint32_t* __restrict__ gz, int k) {
#pragma unroll
    for (int j = 0; j < D; j++) s[j] = gz[GRAY_STRIDE * k + j];
  }
  // element loops: read row 1 ahead of step 0, then at step k >= 1 take the
  // row read one step earlier and read row k + 1 (clamped to the table: at
  // the last step of a 2^13-point block, k + 1 = GRAY_ROWS, the row read is
  // not used)
  __device__ inline void ahead(const uint32_t* __restrict__ gz) {
#pragma unroll
    for (int j = 0; j < D; j++) nx[j] = gz[GRAY_STRIDE + j];
  }
  __device__ inline void step(const uint32_t* __restrict__ gz, int k) {
    const int nr = k + 1 < GRAY_ROWS ? k + 1 : GRAY_ROWS - 1;
#pragma unroll
    for (int j = 0; j < D; j++) {
      s[j] = nx[j];
      nx[j] = gz[GRAY_STRIDE * nr + j];
    }
  }
  // called at the end of a step's work: the row read by step() is taken
  // there, so its scalar load is not moved next to its use in the next step
  __device__ inline void hold() {
#pragma unroll
    for (int j = 0; j < D; j++) asm volatile("" : "+s"(nx[j]));
  }
  // unrolled element loops: the same, and no later row read is hoisted
  // above it (all rows read up front exceed the scalar register file)
  __device__ inline void hold_rows() {
#pragma unroll
    for (int j = 0; j < D; j++) asm volatile("" : "+s"(nx[j])::"memory");
  }
  __device__ inline uint32_t u(int j) const { return a[j] ^ s[j]; }
};

// Order-2 DSI kernel in integer-scaled form.  With X = u (the digit as an
// integer, exact in FP64) and K2(x) = 3/2 - (5/2) t1(x) - beta(x) x,
//   kappa = 2^32 K2 = (3/2) 2^32 - beta X - (5/2) lead(X),
// where lead(X) = 2^32 t1(x) keeps X's exponent and drops its mantissa, and
// beta X = (r + 1) X with r = find-first-bit-high(u) (-1 for u = 0).  kappa
// is exact in FP64 (dyadic, < 2^53); for u = 0, lead is taken as the
// smallest normal number times 5/4, which vanishes in the subtraction.
template <typename Real> __device__ inline Real dsi2_kappa(uint32_t u);
template <> __device__ inline double dsi2_kappa<double>(uint32_t u) {
  const double X = (double)u;
  int r;
  asm("v_ffbh_u32 %0, %1" : "=v"(r) : "v"(u));
  const double L = __hiloint2double((__double2hiint(X) & 0x7ff00000) + 0x00140000, 0);
  return fma(-(double)r, X, (6442450944.0 - L) - X);
}
template <> __device__ inline float dsi2_kappa<float>(uint32_t u) {
  const float X = __uint2float_rz(u);  // truncation keeps lead(X) = lead(u)
  int r;
  asm("v_ffbh_u32 %0, %1" : "=v"(r) : "v"(u));
  const float L = __int_as_float((__float_as_int(X) & 0x7f800000) + 0x00a00000);
  return fmaf(-(float)r, X, (6442450944.0f - L) - X);
}

// univariate kernel value of a compile-time kernel type
template <typename Real, int KT>
__device__ inline Real kval(uint32_t u, const Params* __restrict__ P);

// The kernel factor of one dimension in scaled form: eta K(u) = s kappa(u),
// so f = 1 + eta K = fma(s, kappa, 1) and derivative sums can accumulate
// kappa and be scaled by s once at the end.  Order 2 uses the integer form
// above (s = eta 2^-32); the other kernels use kappa = K, s = eta.
template <typename Real, int KT>
__device__ inline Real kscale(Real eta) {
  if constexpr (KT == KT_DSI2) return eta * (Real)0x1p-32;
  else return eta;
}
template <typename Real, int KT>
__device__ inline Real kappa(uint32_t u, const Params* __restrict__ P) {
  if constexpr (KT == KT_DSI2) return dsi2_kappa<Real>(u);
  else return kval<Real, KT>(u, P);
}

// The order-2 factor through a 33-entry table indexed by r + 1 (r =
// find-first-bit-high(u), -1 for u = 0): tab[0] = {(3/2) 2^32, 0} and
// tab[r + 1] = {(3/2) 2^32 - (5/2) 2^(31 - r), -(r + 1)}, so that
// kappa = fma(tab.m, X, tab.c).  Every term is a multiple of 1/2 below 2^53,
// so this equals dsi2_kappa<double> exactly, in 4 vector instructions and
// one LDS read instead of 8 instructions.
struct __align__(16) Kap2Entry {
  double c, m;
};
// (An 8-byte table of c alone, with the slope converted from r, measured
// slower: the kernels are bound by VALU issue, not by these LDS reads.)
__device__ inline void fill_kap2_table(Kap2Entry* tab) {
  for (int i = threadIdx.x; i < 33; i += blockDim.x)
    tab[i] = i == 0 ? Kap2Entry{6442450944.0, 0.0}
                    : Kap2Entry{6442450944.0 - 2.5 * ldexp(1.0, 32 - i), -(double)i};
}
__device__ inline double dsi2_kappa_tab(uint32_t u, const Kap2Entry* tab) {
  int r;
  asm("v_ffbh_u32 %0, %1" : "=v"(r) : "v"(u));
  const Kap2Entry e = tab[r + 1];
  return fma(e.m, (double)u, e.c);
}
// kernel types whose FP64 factor uses the table
template <typename Real, int KT>
constexpr bool uses_kap2_table() {
  return KT == KT_DSI2 && sizeof(Real) == 8;
}
template <typename Real, int KT>
__device__ inline Real kappa_t(uint32_t u, const Params* __restrict__ P, const Kap2Entry* tab) {
  if constexpr (uses_kap2_table<Real, KT>()) return dsi2_kappa_tab(u, tab);
  else return kappa<Real, KT>(u, P);
}

template <typename Real, int KT>
__device__ inline Real kval(uint32_t u, const Params* __restrict__ P) {
  if constexpr (KT == KT_DSIA) {
    Real k[4];
    dsi_khat_all<Real>(u, k);
    return RT<Real>::bw(P, 0) * k[0] + RT<Real>::bw(P, 1) * k[1] + RT<Real>::bw(P, 2) * k[2] +
           RT<Real>::bw(P, 3) * k[3];
  } else if constexpr (KT >= KT_SI1) {
    return si_kern<Real>(KT - 10, u);
  } else {
    return dsi_khat_o<Real, KT>(u);
  }
}

// Walsh-Hadamard butterflies over the E register slots of a thread (slot e
// holds in-block index t + 256 e, so these are the index bits 8 ..).
template <typename Real, int E>
__device__ inline void reg_fwht(Real (&v)[E]) {
#pragma unroll
  for (int h = 1; h < E; h <<= 1) {
#pragma unroll
    for (int k = 0; k < E; k++) {
      if (!(k & h)) {
        const Real a = v[k], b = v[k + h];
        v[k] = a + b;
        v[k + h] = a - b;
      }
    }
  }
}

// Dimension slots are padded to D (padding slots carry eta = 0, so their
// kernel factor is exactly 1): D in {2, 4, 6, 8, 10, 12, 16, 32}.
#define MTGP_DISPATCH_D(d, MACRO, ...)          \
  do {                                          \
    if ((d) <= 2) MACRO(2, __VA_ARGS__);        \
    else if ((d) <= 4) MACRO(4, __VA_ARGS__);   \
    else if ((d) <= 6) MACRO(6, __VA_ARGS__);   \
    else if ((d) <= 8) MACRO(8, __VA_ARGS__);   \
    else if ((d) <= 10) MACRO(10, __VA_ARGS__); \
    else if ((d) <= 12) MACRO(12, __VA_ARGS__); \
    else if ((d) <= 16) MACRO(16, __VA_ARGS__); \
    else MACRO(32, __VA_ARGS__);                \
  } while (0)

}  // namespace mtgp

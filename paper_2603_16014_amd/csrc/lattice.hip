// Shifted rank-1 lattices with shift-invariant kernels (Condition "Fast
// MTGP", SI-LAT): V^dagger a = n^-1/2 F (bit reversal of a) (Theorem "Fast
// GP computations"), so kernel columns are taken in natural lattice order
// j (point j g / n + shift) and transformed by the unnormalised DFT
// F_fj = e^{-2 pi i f j / n}.
//
// Forward: radix-2 decimation in frequency over all m index bits, natural
// input, bit-reversed output, so the spectrum holds frequency f at position
// bitrev_m(f) (frequency 0 at position 0; the per-frequency algebra does not
// care about the order, and the data transform uses the same layout).  The
// stages of the high index bits run first, in register passes of 5 bits (4
// where the bit count asks for it): a thread owns the 2^hb values strided by
// 2^lo that share its low index, so every load and store of a wave is 64
// consecutive elements.  The twiddle of the stage of bit k = lo + s on the
// pair of register slot r (r < 2^s) is
//   e^{-i pi (low + r 2^lo) / 2^k} = e^{-i pi low / 2^k} e^{-i pi r / 2^s},
// a per-thread base (one sincospi per pass, squared down the stages) times a
// constant.  Two adjacent 5-bit passes can run as one tile pass (8 columns x
// 2^10 rows through LDS, each element read and written once for both).  The
// first pass generates the kernel column (or loads the data) itself; the low
// L in [8, 10] bits finish in a wave-level pass.
// Adjoint: u(j) = Re sum_f omega(f) e^{-2 pi i f j / n} from omega stored at
// bit-reversed positions is the transposed network, decimation in time: the
// wave pass over the low bits first, then the register (or tile) passes
// upwards, the last one fused with the derivative reduction of the
// regenerated column (or with storing Re in natural order).
#include <cmath>

#include "colgen.h"

#include "latdev.h"

namespace mtgp {

template <typename R>
__device__ inline cx<R> cmul(cx<R> a, cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ inline cx<R> cadd(cx<R> a, cx<R> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename R>
__device__ inline cx<R> csub(cx<R> a, cx<R> b) {
  return {a.x - b.x, a.y - b.y};
}
template <typename R>
__device__ inline cx<R> to_cx(cx<double> a) {
  return {(R)a.x, (R)a.y};
}

// e^{-i pi k / 2^e}, FP64 (the angle is an exact dyadic)
__device__ inline cx<double> expmpi(int64_t k, int e) {
  double s, c;
  sincospi(-ldexp((double)k, -e), &s, &c);
  return {c, s};
}

__device__ inline int64_t bitrev64(int64_t p, int L) {
  return L ? (int64_t)(__brevll((unsigned long long)p) >> (64 - L)) : 0;
}

// e^{-i pi t / 16}, t < 16: the constant factors of the register passes
struct LatTab {
  double c[16], s[16];
};
static LatTab lat_tab() {
  constexpr double kPi = 3.14159265358979323846;
  LatTab t;
  for (int k = 0; k < 16; k++) {
    t.c[k] = std::cos(kPi * k / 16.0);
    t.s[k] = -std::sin(kPi * k / 16.0);
  }
  t.c[0] = 1.0;
  t.s[0] = 0.0;
  t.c[8] = 0.0;
  t.s[8] = -1.0;
  return t;
}

// tw[k] = e^{-i pi k / 2^(L-1)}, k < 2^(L-1), from <= 32 fine and <= 64
// coarse factors (tmp holds >= 96 entries); ends with a barrier.
template <typename R>
__device__ inline void fill_twiddles(cx<R>* tw, int L, cx<double>* tmp) {
  if (L > 0) {
    const int h = L - 1;
    const int fb = h < 5 ? h : 5, nf = 1 << fb, nc = 1 << (h - fb);
    for (int k = threadIdx.x; k < nf + nc; k += blockDim.x)
      tmp[k] = k < nf ? expmpi(k, h) : expmpi((int64_t)(k - nf) << fb, h);
    __syncthreads();
    for (int k = threadIdx.x; k < (1 << h); k += blockDim.x)
      tw[k] = to_cx<R>(cmul<double>(tmp[nf + (k >> fb)], tmp[k & (nf - 1)]));
  }
  __syncthreads();
}

// In-LDS radix-2 DIF over the L low bits of one contiguous block (natural in,
// bit-reversed out; the twiddles of these stages depend on the low bits only).
template <typename R>
__device__ inline void lds_dif(cx<R>* a, int L, int stride, const cx<R>* tw) {
  const int hb = L - 1;
  for (int s = L - 1; s >= 0; s--) {
    const int half = 1 << s;
    for (int g = threadIdx.x; g < (1 << hb); g += blockDim.x) {
      const int k = g & (half - 1);
      const int i = ((g >> s) << (s + 1)) | k;
      cx<R>* pa = a + lds_at(0, stride, i);
      cx<R>* pb = a + lds_at(0, stride, i + half);
      const cx<R> A = *pa, B = *pb;
      *pa = cadd(A, B);
      *pb = cmul<R>(csub(A, B), tw[k << (hb - s)]);
    }
    __syncthreads();
  }
}

// In-LDS radix-2 DIT over the L low bits (bit-reversed in, natural out).
template <typename R>
__device__ inline void lds_dit(cx<R>* a, int L, int stride, const cx<R>* tw) {
  const int hb = L - 1;
  for (int s = 0; s < L; s++) {
    const int half = 1 << s;
    for (int g = threadIdx.x; g < (1 << hb); g += blockDim.x) {
      const int k = g & (half - 1);
      const int i = ((g >> s) << (s + 1)) | k;
      cx<R>* pa = a + lds_at(0, stride, i);
      cx<R>* pb = a + lds_at(0, stride, i + half);
      const cx<R> A = *pa, B = cmul<R>(*pb, tw[k << (hb - s)]);
      *pa = cadd(A, B);
      *pb = csub(A, B);
    }
    __syncthreads();
  }
}

enum { SRC_GEN = LAT_SRC_GEN, SRC_Y = LAT_SRC_Y, SRC_X = LAT_SRC_X, SRC_WORK = 3 };
enum { SINK_WORK = LAT_SINK_Z, SINK_REDUCE = LAT_SINK_REDUCE, SINK_REAL = LAT_SINK_REAL };

// real input of the forward transform at natural index j of vector v: the
// kernel column (SRC_GEN), y[bitrev_m(j)] (SRC_Y) or y[j] (SRC_X)
template <typename CR, int SRC, int KT>
__device__ inline CR src_value(const void* y, int y_f32, int v, uint32_t j, int m,
                               const uint32_t* __restrict__ gen,
                               const uint32_t* __restrict__ colshift,
                               const Params* __restrict__ P, int d) {
  if constexpr (SRC == SRC_GEN) {
    return lat_col_value<CR, KT>(gen, colshift + (size_t)v * d, d, j, m, P);
  } else {
    const size_t idx = (size_t)v * ((size_t)1 << m) +
                       (SRC == SRC_Y ? (size_t)bitrev64((int64_t)j, m) : (size_t)j);
    return y_f32 ? (CR) static_cast<const float*>(y)[idx] : (CR) static_cast<const double*>(y)[idx];
  }
}

// ---------------------------------------------------------------------------
// radix-2^HB butterflies of one register pass over the bits [lo, lo + HB)
// on the 2^HB values a[r] (row r at index low + (r << lo)) that share the
// index `low` below lo.  The twiddle of the stage at bit lo + s is
// e^{-i pi low / 2^(lo+s)} (a per-thread base, squared from stage to stage)
// times e^{-i pi (r mod 2^s) / 2^s} (constant table).
// ---------------------------------------------------------------------------
template <typename CR, int HB>
__device__ inline void dif_regs(cx<CR> (&a)[1 << HB], const LatTab& tab, int64_t low, int lo) {
  constexpr int R = 1 << HB;
  cx<double> B = expmpi(low, lo + HB - 1);
#pragma unroll
  for (int s = HB - 1; s >= 0; s--) {
    const cx<CR> b = to_cx<CR>(B);
#pragma unroll
    for (int r = 0; r < R; r++) {
      if (!(r & (1 << s))) {
        const int t = (r & ((1 << s) - 1)) << (4 - s);
        const cx<CR> w = t == 0 ? b : cmul<CR>(b, {(CR)tab.c[t], (CR)tab.s[t]});
        const cx<CR> A = a[r], C = a[r + (1 << s)];
        a[r] = cadd(A, C);
        a[r + (1 << s)] = cmul<CR>(csub(A, C), w);
      }
    }
    B = cmul<double>(B, B);
  }
}

// the transpose (decimation in time, stages from bit lo upwards)
template <typename CR, int HB>
__device__ inline void dit_regs(cx<CR> (&a)[1 << HB], const LatTab& tab, int64_t low, int lo) {
  constexpr int R = 1 << HB;
  cx<double> Bs[HB];
  Bs[HB - 1] = expmpi(low, lo + HB - 1);
#pragma unroll
  for (int s = HB - 2; s >= 0; s--) Bs[s] = cmul<double>(Bs[s + 1], Bs[s + 1]);
#pragma unroll
  for (int s = 0; s < HB; s++) {
    const cx<CR> b = to_cx<CR>(Bs[s]);
#pragma unroll
    for (int r = 0; r < R; r++) {
      if (!(r & (1 << s))) {
        const int t = (r & ((1 << s) - 1)) << (4 - s);
        const cx<CR> w = t == 0 ? b : cmul<CR>(b, {(CR)tab.c[t], (CR)tab.s[t]});
        const cx<CR> A = a[r], C = cmul<CR>(a[r + (1 << s)], w);
        a[r] = cadd(A, C);
        a[r + (1 << s)] = csub(A, C);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// register passes over the bits [lo, lo + HB): grid (2^(m - HB - 8), nvec),
// 256 threads; block x covers 256 consecutive low indices of one high index
// ---------------------------------------------------------------------------
// (ublk: the block-uniform part of the index, low: the thread's low index;
// element r of the thread sits at ublk + (r << lo) + threadIdx.x)
struct RegIdx {
  int64_t low, ublk;
  __device__ inline RegIdx(int lo, int HB) {
    const int gb = lo - 8;
    const int64_t grp = blockIdx.x & (((int64_t)1 << gb) - 1);
    const int64_t hi = (int64_t)blockIdx.x >> gb;
    low = (grp << 8) + threadIdx.x;
    ublk = (hi << (lo + HB)) + (grp << 8);
  }
  __device__ inline int64_t at(int r, int lo) const { return ublk + ((int64_t)r << lo) + threadIdx.x; }
};

// BUF: the rows of a block are read and written through raw buffer
// resources over its window of 2^(lo + HB) elements (below 2^31 bytes), one
// scalar offset per row instead of a 64-bit vector address per row.
template <typename CR, typename TOut, int HB, int SRC, int KT, bool BUF>
__global__ __launch_bounds__(256) void lat_dif_reg_kernel(
    const LatTab tab, cx<CR>* __restrict__ work, cx<TOut>* __restrict__ out, int64_t vstride,
    int m, int lo, const void* __restrict__ y, int y_f32, const uint32_t* __restrict__ gen,
    const uint32_t* __restrict__ colshift, const Params* __restrict__ P, int d) {
  constexpr int R = 1 << HB;
  static_assert(HB >= 1 && HB <= 5, "constant twiddles cover 5 bits");
  const int v = blockIdx.y;
  const RegIdx ix(lo, HB);
  const int64_t vb = (int64_t)v * vstride + ix.ublk;
  cx<CR> a[R];
  if constexpr (SRC == SRC_GEN) {
    // c(j) = gamma prod_q (1 + eta_q K_q(j)), dimensions outside: the digit
    // of element r advances by the constant step(2^lo) from element 0
    CR c[R];
#pragma unroll
    for (int r = 0; r < R; r++) c[r] = RT<CR>::gamma(P);
    const uint32_t* sh = colshift + (size_t)v * d;
    const uint32_t i0 = (uint32_t)ix.at(0, lo);
    for (int q = 0; q < d; q++) {
      SiFactor<CR, KT> fk;
      fk.init(RT<CR>::eta(P, q));
      uint32_t u = lat_z(gen[q], i0, m) + sh[q];
      const uint32_t step = lat_z(gen[q], 1u << lo, m);
#pragma unroll
      for (int r = 0; r < R; r++) {
        c[r] = fma(c[r], fk.eta_k(u), c[r]);
        u += step;
      }
    }
#pragma unroll
    for (int r = 0; r < R; r++) a[r] = {c[r], (CR)0};
  } else {
#pragma unroll
    for (int r = 0; r < R; r++) {
      const int64_t i = ix.at(r, lo);
      if constexpr (SRC == SRC_WORK && BUF)
        a[r] = buf_load<cx<CR>>(buf_rsrc(work + vb, (int)(sizeof(cx<CR>) << (lo + HB))),
                                threadIdx.x * (uint32_t)sizeof(cx<CR>),
                                ((uint32_t)r << lo) * (uint32_t)sizeof(cx<CR>));
      else if constexpr (SRC == SRC_WORK)
        a[r] = (work + vb + ((int64_t)r << lo))[threadIdx.x];
      else
        a[r] = {src_value<CR, SRC, KT>(y, y_f32, v, (uint32_t)i, m, gen, colshift, P, d), (CR)0};
    }
  }
  dif_regs<CR, HB>(a, tab, ix.low, lo);
#pragma unroll
  for (int r = 0; r < R; r++) {
    const cx<TOut> o = {(TOut)a[r].x, (TOut)a[r].y};
    if constexpr (BUF)
      buf_store<cx<TOut>>(o, buf_rsrc(out + vb, (int)(sizeof(cx<TOut>) << (lo + HB))),
                          threadIdx.x * (uint32_t)sizeof(cx<TOut>),
                          ((uint32_t)r << lo) * (uint32_t)sizeof(cx<TOut>));
    else
      (out + vb + ((int64_t)r << lo))[threadIdx.x] = o;
  }
}

// SINK_WORK: store back to work; SINK_REAL: real_out[v][j] = Re * scale;
// SINK_REDUCE: derivative sums (Re values staged in dynamic LDS, R x 256 CR).
template <typename CR, int HB, int SINK, int KT, int D, bool BUF>
__global__ __launch_bounds__(256) void lat_dit_reg_kernel(
    const LatTab tab, cx<CR>* __restrict__ work, double* __restrict__ real_out, int64_t vstride,
    int m, int lo, double scale, const uint32_t* __restrict__ gen,
    const uint32_t* __restrict__ colshift, const Params* __restrict__ P, int d,
    double* __restrict__ partials) {
  constexpr int R = 1 << HB;
  static_assert(HB >= 1 && HB <= 5, "constant twiddles cover 5 bits");
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[4 * (D + 1)];
  const int v = blockIdx.y;
  const RegIdx ix(lo, HB);
  const int64_t vb = (int64_t)v * vstride + ix.ublk;
  const int nb = (int)(sizeof(cx<CR>) << (lo + HB));
  constexpr uint32_t cb = sizeof(cx<CR>);
  cx<CR> a[R];
#pragma unroll
  for (int r = 0; r < R; r++) {
    if constexpr (BUF)
      a[r] = buf_load<cx<CR>>(buf_rsrc(work + vb, nb), threadIdx.x * cb, ((uint32_t)r << lo) * cb);
    else
      a[r] = (work + vb + ((int64_t)r << lo))[threadIdx.x];
  }
  dit_regs<CR, HB>(a, tab, ix.low, lo);
  if constexpr (SINK == SINK_WORK) {
#pragma unroll
    for (int r = 0; r < R; r++) {
      if constexpr (BUF)
        buf_store<cx<CR>>(a[r], buf_rsrc(work + vb, nb), threadIdx.x * cb, ((uint32_t)r << lo) * cb);
      else
        (work + vb + ((int64_t)r << lo))[threadIdx.x] = a[r];
    }
  } else if constexpr (SINK == SINK_REAL) {
#pragma unroll
    for (int r = 0; r < R; r++)
      (real_out + ((size_t)v << m) + ix.ublk + ((int64_t)r << lo))[threadIdx.x] =
          (double)a[r].x * scale;
  } else {
    CR* stage = reinterpret_cast<CR*>(smem);
#pragma unroll
    for (int r = 0; r < R; r++) stage[r * 256 + threadIdx.x] = a[r].x;
    // each thread reads back only its own slots: no barrier needed
    LatReduce<CR, KT, D> lr;
    lr.init(gen, colshift + (size_t)v * d, d, P, (uint32_t)ix.at(0, lo), 1u << lo, m);
#pragma unroll 1
    for (int r = 0; r < R; r++) lr.add(stage[r * 256 + threadIdx.x]);
    lr.store(d, red, partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * adj_nq(d));
  }
}

// ---------------------------------------------------------------------------
// tile passes: the two top 5-bit register passes, bits [lo, lo + 10), in one
// pass.  A block takes the 8 adjacent low indices j0 .. j0 + 7 (runs of 128
// bytes per row) over all 1024 rows hi = h1 + 32 h2 (h1: bits lo .. lo + 4,
// h2: bits lo + 5 .. lo + 9).  Phase 1: thread (c, h1) runs the pass over
// h2 on its 32 rows (the index below lo + 5 is j0 + c + (h1 << lo)); the
// values go through an LDS tile; phase 2: thread (c, h2) runs the pass over
// h1 (index below lo: j0 + c).  The arithmetic is that of the two register
// passes; the HBM traffic of one.  Grid (2^(m - 13), nvec): 2^(lo - 3) column
// groups times the 2^(m - lo - 10) values of the index above lo + 10; 256 threads,
// dynamic LDS lat_tile_lds_bytes; rows through raw buffer resources over a
// window of 2^(lo + 10) elements (below 2^30 bytes).
// ---------------------------------------------------------------------------
constexpr int kTileKC = 8, kTileR = 32, kTilePad = kTileKC;
__host__ __device__ inline int tile_at(int hi, int c) {
  // one run of padding per 32 rows keeps a phase-2 access on distinct banks
  return hi * kTileKC + c + (hi >> 5) * kTilePad;
}
static size_t lat_tile_lds_bytes(size_t cbytes) {
  return ((size_t)kTileR * kTileR * kTileKC + (size_t)kTileR * kTilePad) * cbytes;
}

template <typename CR, int SRC, int KT>
__global__ __launch_bounds__(256) void lat_dif_tile_kernel(
    const LatTab tab, cx<CR>* __restrict__ work, int64_t vstride, int m, int lo,
    const void* __restrict__ y, int y_f32, const uint32_t* __restrict__ gen,
    const uint32_t* __restrict__ colshift, const Params* __restrict__ P, int d) {
  extern __shared__ __align__(16) unsigned char smem[];
  cx<CR>* tile = reinterpret_cast<cx<CR>*>(smem);
  const int v = blockIdx.y;
  // block x: column group (the low lo - 3 bits) and the index above lo + 10
  const int cgb = lo - 3;
  const int64_t j0 = (int64_t)(blockIdx.x & ((1u << cgb) - 1)) * kTileKC;
  const int64_t hiw = ((int64_t)blockIdx.x >> cgb) << (lo + 10);
  const int c = threadIdx.x & (kTileKC - 1), h = threadIdx.x >> 3;
  constexpr uint32_t cb = sizeof(cx<CR>);
  const __amdgpu_buffer_rsrc_t rw =
      buf_rsrc(work + (int64_t)v * vstride + hiw + j0, (int)(cb << (lo + 10)));
  cx<CR> a[kTileR];
  // phase 1: thread (c, h1 = h), rows h2 = r at index hiw + low1 + (r << (lo + 5))
  {
    const int64_t low1 = j0 + c + ((int64_t)h << lo);
    if constexpr (SRC == SRC_GEN) {
      CR cv[kTileR];
#pragma unroll
      for (int r = 0; r < kTileR; r++) cv[r] = RT<CR>::gamma(P);
      const uint32_t* sh = colshift + (size_t)v * d;
      for (int q = 0; q < d; q++) {
        SiFactor<CR, KT> fk;
        fk.init(RT<CR>::eta(P, q));
        uint32_t u = lat_z(gen[q], (uint32_t)(hiw + low1), m) + sh[q];
        const uint32_t step = lat_z(gen[q], 1u << (lo + 5), m);
#pragma unroll
        for (int r = 0; r < kTileR; r++) {
          cv[r] = fma(cv[r], fk.eta_k(u), cv[r]);
          u += step;
        }
      }
#pragma unroll
      for (int r = 0; r < kTileR; r++) a[r] = {cv[r], (CR)0};
    } else {
#pragma unroll
      for (int r = 0; r < kTileR; r++)
        a[r] = {src_value<CR, SRC, KT>(y, y_f32, v,
                                       (uint32_t)(hiw + low1 + ((int64_t)r << (lo + 5))), m, gen,
                                       colshift, P, d),
                (CR)0};
    }
    dif_regs<CR, 5>(a, tab, low1, lo + 5);
#pragma unroll
    for (int r = 0; r < kTileR; r++) tile[tile_at(h + kTileR * r, c)] = a[r];
  }
  __syncthreads();
  // phase 2: thread (c, h2 = h), rows h1 = r
#pragma unroll
  for (int r = 0; r < kTileR; r++) a[r] = tile[tile_at(r + kTileR * h, c)];
  dif_regs<CR, 5>(a, tab, j0 + c, lo);
#pragma unroll
  for (int r = 0; r < kTileR; r++)  // lane part in the vector offset, row part scalar
    buf_store<cx<CR>>(a[r], rw, ((uint32_t)c + ((uint32_t)h << (lo + 5))) * cb,
                      ((uint32_t)r << lo) * cb);
}

// Adjoint: phase 1 runs the DIT pass over h1 (bits lo .. lo + 4), phase 2 the
// one over h2 and the sink: SINK_WORK stores, SINK_REAL writes Re * scale,
// SINK_REDUCE accumulates the derivative sums (one partial row per block).
template <typename CR, int SINK, int KT, int D>
__global__ __launch_bounds__(256) void lat_dit_tile_kernel(
    const LatTab tab, cx<CR>* __restrict__ work, double* __restrict__ real_out, int64_t vstride,
    int m, int lo, double scale, const uint32_t* __restrict__ gen,
    const uint32_t* __restrict__ colshift, const Params* __restrict__ P, int d,
    double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[4 * (D + 1)];
  cx<CR>* tile = reinterpret_cast<cx<CR>*>(smem);
  const int v = blockIdx.y;
  // block x: column group (the low lo - 3 bits) and the index above lo + 10
  const int cgb = lo - 3;
  const int64_t j0 = (int64_t)(blockIdx.x & ((1u << cgb) - 1)) * kTileKC;
  const int64_t hiw = ((int64_t)blockIdx.x >> cgb) << (lo + 10);
  const int c = threadIdx.x & (kTileKC - 1), h = threadIdx.x >> 3;
  constexpr uint32_t cb = sizeof(cx<CR>);
  const __amdgpu_buffer_rsrc_t rw =
      buf_rsrc(work + (int64_t)v * vstride + hiw + j0, (int)(cb << (lo + 10)));
  cx<CR> a[kTileR];
  // phase 1: thread (c, h2 = h), rows h1 = r
#pragma unroll
  for (int r = 0; r < kTileR; r++)  // lane part in the vector offset, row part scalar
    a[r] = buf_load<cx<CR>>(rw, ((uint32_t)c + ((uint32_t)h << (lo + 5))) * cb,
                            ((uint32_t)r << lo) * cb);
  dit_regs<CR, 5>(a, tab, j0 + c, lo);
#pragma unroll
  for (int r = 0; r < kTileR; r++) tile[tile_at(r + kTileR * h, c)] = a[r];
  __syncthreads();
  // phase 2: thread (c, h1 = h), rows h2 = r at index low1 + (r << (lo + 5))
  const int64_t low1 = j0 + c + ((int64_t)h << lo);
#pragma unroll
  for (int r = 0; r < kTileR; r++) a[r] = tile[tile_at(h + kTileR * r, c)];
  dit_regs<CR, 5>(a, tab, low1, lo + 5);
  if constexpr (SINK == SINK_WORK) {
#pragma unroll
    for (int r = 0; r < kTileR; r++)
      buf_store<cx<CR>>(a[r], rw, ((uint32_t)c + ((uint32_t)h << lo)) * cb,
                        ((uint32_t)r << (lo + 5)) * cb);
  } else if constexpr (SINK == SINK_REAL) {
#pragma unroll
    for (int r = 0; r < kTileR; r++)
      real_out[((size_t)v << m) + hiw + low1 + ((int64_t)r << (lo + 5))] = (double)a[r].x * scale;
  } else {
    // the thread rewrites only the tile slots it read, so no barrier
    CR* stage = reinterpret_cast<CR*>(smem);
#pragma unroll
    for (int r = 0; r < kTileR; r++) stage[2 * tile_at(h + kTileR * r, c)] = a[r].x;
    LatReduce<CR, KT, D> lr;
    lr.init(gen, colshift + (size_t)v * d, d, P, (uint32_t)(hiw + low1), 1u << (lo + 5), m);
#pragma unroll 1
    for (int r = 0; r < kTileR; r++) lr.add(stage[2 * tile_at(h + kTileR * r, c)]);
    lr.store(d, red, partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * adj_nq(d));
  }
}

// ---------------------------------------------------------------------------
// LDS passes over the low L bits: grid (2^(m - L), nvec), one contiguous
// block of 2^L each; dynamic LDS = lat_lds_bytes(L)
// ---------------------------------------------------------------------------
// Forward: input from work (SRC_WORK) or generated / loaded (only pass),
// output at the same positions into out, times scale; natural != 0 (only
// pass of the standalone transform) writes position p to bitrev_L(p).
template <typename CR, typename TOut, int SRC, int KT>
__global__ __launch_bounds__(256) void lat_dif_lds_kernel(
    const cx<CR>* __restrict__ work, cx<TOut>* __restrict__ out, int64_t vstride, int m, int L,
    double scale, int natural, const void* __restrict__ y, int y_f32,
    const uint32_t* __restrict__ gen, const uint32_t* __restrict__ colshift,
    const Params* __restrict__ P, int d) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ cx<double> tmp[96];
  const int nb = 1 << L;
  const int stride = lds_stride(L);
  cx<CR>* a = reinterpret_cast<cx<CR>*>(smem);
  cx<CR>* tw = a + stride;
  const int v = blockIdx.y;
  const int64_t b0 = (int64_t)blockIdx.x << L;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    cx<CR> val;
    if constexpr (SRC == SRC_WORK)
      val = work[(size_t)v * vstride + b0 + i];
    else
      val = {src_value<CR, SRC, KT>(y, y_f32, v, (uint32_t)(b0 + i), m, gen, colshift, P, d),
             (CR)0};
    a[lds_at(0, stride, i)] = val;
  }
  fill_twiddles<CR>(tw, L, tmp);
  lds_dif<CR>(a, L, stride, tw);
  for (int p = threadIdx.x; p < nb; p += blockDim.x) {
    const cx<CR> val = a[lds_at(0, stride, p)];
    const int64_t q = natural ? bitrev64(p, L) : p;
    out[(size_t)v * vstride + b0 + q] = {(TOut)(val.x * (CR)scale), (TOut)(val.y * (CR)scale)};
  }
}

// Adjoint: omega (conjugated if conj_in) at its positions, DIT, then
// SINK_WORK (register passes follow), SINK_REAL or SINK_REDUCE (only pass).
template <typename CR, typename TIn, int SINK, int KT, int D>
__global__ __launch_bounds__(256) void lat_dit_lds_kernel(
    const cx<TIn>* __restrict__ spec, cx<CR>* __restrict__ work, double* __restrict__ real_out,
    int64_t vstride, int m, int L, int conj_in, double scale, const uint32_t* __restrict__ gen,
    const uint32_t* __restrict__ colshift, const Params* __restrict__ P, int d,
    double* __restrict__ partials) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ cx<double> tmp[96];
  __shared__ double red[4 * (D + 1)];
  const int nb = 1 << L;
  const int stride = lds_stride(L);
  cx<CR>* a = reinterpret_cast<cx<CR>*>(smem);
  cx<CR>* tw = a + stride;
  const int v = blockIdx.y;
  const int64_t b0 = (int64_t)blockIdx.x << L;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    const cx<TIn> w = spec[(size_t)v * vstride + b0 + i];
    a[lds_at(0, stride, i)] = {(CR)w.x, conj_in ? -(CR)w.y : (CR)w.y};
  }
  fill_twiddles<CR>(tw, L, tmp);
  lds_dit<CR>(a, L, stride, tw);
  if constexpr (SINK == SINK_WORK) {
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
      work[(size_t)v * vstride + b0 + i] = a[lds_at(0, stride, i)];
  } else if constexpr (SINK == SINK_REAL) {
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
      real_out[(size_t)v * ((size_t)1 << m) + b0 + i] = (double)a[lds_at(0, stride, i)].x * scale;
  } else {
    LatReduce<CR, KT, D> lr;
    lr.init(gen, colshift + (size_t)v * d, d, P, (uint32_t)(b0 + threadIdx.x), blockDim.x, m);
    for (int i = threadIdx.x; i < nb; i += blockDim.x) lr.add(a[lds_at(0, stride, i)].x);
    lr.store(d, red, partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * adj_nq(d));
  }
}

// ---------------------------------------------------------------------------
// wave passes over the low L in {8, 9, 10} bits of a multi-pass transform:
// grid (2^(m - L) / 4, nvec), 256 threads; wave w of a block owns the
// sub-block of 2^L consecutive elements 4 blockIdx.x + w and keeps
// E = 2^(L - 6) of them per lane.  Rounds of R = L - 6 bits (the last one
// ragged when R does not divide L) run their radix-2 stages in registers; the
// wave's LDS region re-gathers the values between rounds.  In a round over
// the bits [lo, lo + r), value k = g 2^r + kk of a lane is element
//   (hi << (lo + r)) | (kk << lo) | low,  (hi, low) from q = lane + 64 g,
// so the top round's elements (kk << lo) | lane, and hence the loads of the
// forward and the stores of the adjoint, are coalesced.
// ---------------------------------------------------------------------------
template <int L>
struct WavePass {
  static constexpr int R = L - 6, E = 1 << R;
  static constexpr int NR = (L + R - 1) / R;  // rounds
  // forward rounds from the top: bits [max(hi - R, 0), hi), hi = L - R q;
  // adjoint rounds from the bottom: bits [R q, min(R q + R, L))
  __device__ static inline int dif_lo(int q) { return L - R * q - R > 0 ? L - R * q - R : 0; }
  __device__ static inline int dif_bits(int q) { return L - R * q - dif_lo(q); }
  __device__ static inline int dit_lo(int q) { return R * q; }
  __device__ static inline int dit_bits(int q) { return L - R * q < R ? L - R * q : R; }
  __device__ static inline int elem(int lane, int k, int lo, int r) {
    const int g = k >> r, kk = k & ((1 << r) - 1);
    const int q = lane + 64 * g;
    const int low = q & ((1 << lo) - 1), hi = q >> lo;
    return (hi << (lo + r)) | (kk << lo) | low;
  }
};

// The decimation-in-frequency rounds of one wave's 2^L-element group: the
// group is read from `in` in the first round and left in the wave's LDS
// region `sub` (position i: storage index i of the group), each round ending
// with a block barrier.
template <typename CR, int L>
__device__ inline void wave_dif_rounds(const cx<CR>* __restrict__ in, cx<CR>* sub,
                                       const cx<CR>* tw, int lane, int stride) {
  using WP = WavePass<L>;
  constexpr int E = WP::E, R = WP::R;
  cx<CR> v[E];
  for (int q = 0; q < WP::NR; q++) {
    const int lo = WP::dif_lo(q), r = WP::dif_bits(q);
#pragma unroll
    for (int k = 0; k < E; k++) {
      const int i = WP::elem(lane, k, lo, r);
      v[k] = q == 0 ? in[i] : sub[lds_at(0, stride, i)];
    }
#pragma unroll
    for (int sb = R - 1; sb >= 0; sb--) {
      if (sb >= r) continue;
#pragma unroll
      for (int k = 0; k < E; k++) {
        if (k & (1 << sb)) continue;
        const int i = WP::elem(lane, k, lo, r), kb = lo + sb;
        const cx<CR> w = tw[(i & ((1 << kb) - 1)) << (L - 1 - kb)];
        const cx<CR> A = v[k], C = v[k + (1 << sb)];
        v[k] = cadd(A, C);
        v[k + (1 << sb)] = cmul<CR>(csub(A, C), w);
      }
    }
#pragma unroll
    for (int k = 0; k < E; k++) sub[lds_at(0, stride, WP::elem(lane, k, lo, r))] = v[k];
    __syncthreads();
  }
}

template <typename CR, typename SR, int L>
__global__ __launch_bounds__(256) void lat_dif_wave_kernel(const cx<CR>* __restrict__ work,
                                                           cx<SR>* __restrict__ out,
                                                           int64_t vstride, double scale) {
  using WP = WavePass<L>;
  constexpr int E = WP::E;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ cx<double> tmp[96];
  const int stride = lds_stride(L);
  cx<CR>* tw = reinterpret_cast<cx<CR>*>(smem);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  cx<CR>* sub = tw + (1 << (L - 1)) + wv * stride;
  const int64_t b0 = ((int64_t)blockIdx.x * 4 + wv) << L;
  const cx<CR>* in = work + (size_t)blockIdx.y * vstride + b0;
  fill_twiddles<CR>(tw, L, tmp);
  wave_dif_rounds<CR, L>(in, sub, tw, lane, stride);
  cx<SR>* o = out + (size_t)blockIdx.y * vstride + b0;
#pragma unroll
  for (int k = 0; k < E; k++) {
    const cx<CR> val = sub[lds_at(0, stride, lane + 64 * k)];
    o[lane + 64 * k] = {(SR)(val.x * (CR)scale), (SR)(val.y * (CR)scale)};
  }
}

// The same pass writing natural frequency order (the standalone transform of
// a multi-pass length 2^m): a block's NW = 2^B waves take the groups
// g_j = g0 + j 2^(m-L-B), g0 = blockIdx.x, whose bit-reversed indices differ
// in their B lowest bits only: bitrev_{m-L}(g_j) = 2^B bitrev_{m-L-B}(g0) +
// bitrev_B(j).  Position i of group g_j holds frequency
// bitrev_L(i) 2^(m-L) + bitrev_{m-L}(g_j), so for each i the groups fill NW
// consecutive frequencies, and a thread writes slot jj of row i from group
// bitrev_B(jj): one run of NW complex values per row.
template <typename CR, typename SR, int L, int B>
__global__ __launch_bounds__(64 << B) void lat_dif_wave_natural_kernel(
    const cx<CR>* __restrict__ work, cx<SR>* __restrict__ out, int64_t vstride, int m,
    double scale) {
  using WP = WavePass<L>;
  constexpr int E = WP::E, NW = 1 << B;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ cx<double> tmp[96];
  const int stride = lds_stride(L);
  cx<CR>* tw = reinterpret_cast<cx<CR>*>(smem);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  cx<CR>* sub0 = tw + (1 << (L - 1));
  const int gb = m - L - B;  // bits of g0
  const int64_t g = (int64_t)blockIdx.x + ((int64_t)wv << gb);
  const cx<CR>* in = work + (size_t)blockIdx.y * vstride + (g << L);
  fill_twiddles<CR>(tw, L, tmp);
  wave_dif_rounds<CR, L>(in, sub0 + wv * stride, tw, lane, stride);
  // every wave's rounds end with a barrier, so all NW groups are in LDS
  const int64_t base =
      (int64_t)NW * (int64_t)(gb > 0 ? __brev((unsigned)blockIdx.x) >> (32 - gb) : 0);
  cx<SR>* o = out + (size_t)blockIdx.y * vstride + base;
  const int jj = threadIdx.x & (NW - 1);
  const cx<CR>* src = sub0 + (int)(__brev((unsigned)jj) >> (32 - B)) * stride;
#pragma unroll
  for (int k = 0; k < E; k++) {
    const int i = (threadIdx.x >> B) + 64 * k;  // 64 rows per k, NW slots each
    const cx<CR> val = src[lds_at(0, stride, i)];
    const int64_t f = ((int64_t)(__brev((unsigned)i) >> (32 - L)) << (m - L)) + jj;
    o[f] = {(SR)(val.x * (CR)scale), (SR)(val.y * (CR)scale)};
  }
}

template <typename CR, typename SR, int L>
__global__ __launch_bounds__(256) void lat_dit_wave_kernel(const cx<SR>* __restrict__ spec,
                                                           cx<CR>* __restrict__ work,
                                                           int64_t vstride, int conj_in) {
  using WP = WavePass<L>;
  constexpr int E = WP::E, R = WP::R;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ cx<double> tmp[96];
  const int stride = lds_stride(L);
  cx<CR>* tw = reinterpret_cast<cx<CR>*>(smem);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  cx<CR>* sub = tw + (1 << (L - 1)) + wv * stride;
  const int64_t b0 = ((int64_t)blockIdx.x * 4 + wv) << L;
  const cx<SR>* in = spec + (size_t)blockIdx.y * vstride + b0;
#pragma unroll
  for (int k = 0; k < E; k++) {
    const cx<SR> w = in[lane + 64 * k];
    sub[lds_at(0, stride, lane + 64 * k)] = {(CR)w.x, conj_in ? -(CR)w.y : (CR)w.y};
  }
  fill_twiddles<CR>(tw, L, tmp);  // ends with a barrier
  cx<CR> v[E];
  cx<CR>* o = work + (size_t)blockIdx.y * vstride + b0;
  for (int q = 0; q < WP::NR; q++) {
    const int lo = WP::dit_lo(q), r = WP::dit_bits(q);
#pragma unroll
    for (int k = 0; k < E; k++) v[k] = sub[lds_at(0, stride, WP::elem(lane, k, lo, r))];
#pragma unroll
    for (int sb = 0; sb < R; sb++) {
      if (sb >= r) continue;
#pragma unroll
      for (int k = 0; k < E; k++) {
        if (k & (1 << sb)) continue;
        const int i = WP::elem(lane, k, lo, r), kb = lo + sb;
        const cx<CR> w = tw[(i & ((1 << kb) - 1)) << (L - 1 - kb)];
        const cx<CR> A = v[k], C = cmul<CR>(v[k + (1 << sb)], w);
        v[k] = cadd(A, C);
        v[k + (1 << sb)] = csub(A, C);
      }
    }
    if (q + 1 < WP::NR) {
#pragma unroll
      for (int k = 0; k < E; k++) sub[lds_at(0, stride, WP::elem(lane, k, lo, r))] = v[k];
      __syncthreads();
    } else {
#pragma unroll
      for (int k = 0; k < E; k++) o[WP::elem(lane, k, lo, r)] = v[k];
    }
  }
}

static size_t wave_lds_bytes(int L, size_t cbytes) {
  return ((size_t)4 * lds_stride(L) + (1u << (L - 1))) * cbytes;
}

template <typename CR, typename SR>
static void launch_dif_wave(int L, dim3 grid, hipStream_t st, const cx<CR>* work, cx<SR>* spec,
                            int64_t vstride, double scale) {
  const size_t lds = wave_lds_bytes(L, sizeof(cx<CR>));
  if (L == 8)
    hipLaunchKernelGGL((lat_dif_wave_kernel<CR, SR, 8>), grid, dim3(256), lds, st, work, spec,
                       vstride, scale);
  else if (L == 9)
    hipLaunchKernelGGL((lat_dif_wave_kernel<CR, SR, 9>), grid, dim3(256), lds, st, work, spec,
                       vstride, scale);
  else
    hipLaunchKernelGGL((lat_dif_wave_kernel<CR, SR, 10>), grid, dim3(256), lds, st, work, spec,
                       vstride, scale);
}

// groups per block of the natural-order wave pass: runs of 128 bytes of the
// output (8 complex FP64 or 16 complex FP32 values; measured on [29][2^24]:
// FP64 64 / 128 / 256-byte runs 10.6 / 9.8 / 10.1 ms, FP32 64 / 128 bytes
// 6.6 / 6.3 ms per transform), and the block's LDS (one region per group plus
// the twiddles) within 160 KB
template <typename CR, typename SR>
static int wave_natural_bits(int L, int m) {
  int B = sizeof(cx<SR>) >= 16 ? 3 : 4;
  while (B > 0 && (((size_t)lds_stride(L) << B) + (1u << (L - 1))) * sizeof(cx<CR>) > 163840) B--;
  if (B > m - L) B = m - L;
  return B;
}

template <typename CR, typename SR, int B>
static void launch_dif_wave_natural_b(int L, dim3 grid, hipStream_t st, const cx<CR>* work,
                                      cx<SR>* X, int64_t vstride, int m, double scale) {
  const size_t lds = (((size_t)lds_stride(L) << B) + (1u << (L - 1))) * sizeof(cx<CR>);
  const dim3 block(64 << B);
  if (L == 8)
    hipLaunchKernelGGL((lat_dif_wave_natural_kernel<CR, SR, 8, B>), grid, block, lds, st, work,
                       X, vstride, m, scale);
  else if (L == 9)
    hipLaunchKernelGGL((lat_dif_wave_natural_kernel<CR, SR, 9, B>), grid, block, lds, st, work,
                       X, vstride, m, scale);
  else
    hipLaunchKernelGGL((lat_dif_wave_natural_kernel<CR, SR, 10, B>), grid, block, lds, st, work,
                       X, vstride, m, scale);
}

template <typename CR, typename SR>
static void launch_dif_wave_natural(int L, int nvec, hipStream_t st, const cx<CR>* work,
                                    cx<SR>* X, int64_t vstride, int m, double scale) {
  const int B = wave_natural_bits<CR, SR>(L, m);
  const dim3 grid(1u << (m - L - B), nvec);
  switch (B) {
    case 4: launch_dif_wave_natural_b<CR, SR, 4>(L, grid, st, work, X, vstride, m, scale); break;
    case 3: launch_dif_wave_natural_b<CR, SR, 3>(L, grid, st, work, X, vstride, m, scale); break;
    case 2: launch_dif_wave_natural_b<CR, SR, 2>(L, grid, st, work, X, vstride, m, scale); break;
    case 1: launch_dif_wave_natural_b<CR, SR, 1>(L, grid, st, work, X, vstride, m, scale); break;
    default: launch_dif_wave_natural_b<CR, SR, 0>(L, grid, st, work, X, vstride, m, scale); break;
  }
}

template <typename CR, typename SR>
static void launch_dit_wave(int L, dim3 grid, hipStream_t st, const cx<SR>* spec, cx<CR>* work,
                            int64_t vstride, int conj_in) {
  const size_t lds = wave_lds_bytes(L, sizeof(cx<CR>));
  if (L == 8)
    hipLaunchKernelGGL((lat_dit_wave_kernel<CR, SR, 8>), grid, dim3(256), lds, st, spec, work,
                       vstride, conj_in);
  else if (L == 9)
    hipLaunchKernelGGL((lat_dit_wave_kernel<CR, SR, 9>), grid, dim3(256), lds, st, spec, work,
                       vstride, conj_in);
  else
    hipLaunchKernelGGL((lat_dit_wave_kernel<CR, SR, 10>), grid, dim3(256), lds, st, spec, work,
                       vstride, conj_in);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Schedule: m <= 12 is one LDS pass.  Otherwise the low L bits (8..10) go
// through the wave pass and the other bits through as few register passes
// as possible, 5 bits wide where the bits allow and 4 bits for the rest
// (the top passes).  In FP64 a 5-bit pass needs 200-256 VGPRs, 1-2 waves per
// SIMD, but keeps 32 loads in flight per thread, and runs faster than
// 4-bit passes at 3 waves per SIMD, which need one pass more at 2^24.  An
// LDS pass over 11 or 12 low bits (one block of 2^L per vector chunk, L
// radix-2 stages between barriers) measured 4.6 times slower per byte than
// the wave pass, so a 4-bit register pass replaces it where m - 10 is not
// covered by 5-bit passes.
constexpr int kLatHB = 5;  // widest register pass
constexpr int kLatMaxPasses = 5;
struct LatSched {
  int L;                   // LDS / wave-pass bits
  int np;                  // register passes
  int hb[kLatMaxPasses];   // pass q covers the bits [lo(q), lo(q) + hb[q])
  int lo(int q) const {
    int l = L;
    for (int i = 0; i < q; i++) l += hb[i];
    return l;
  }
};
static LatSched lat_sched(int m) {
  LatSched s{};
  if (m <= 12) {
    s.L = m;
    return s;
  }
  s.np = (m - 10 + kLatHB - 1) / kLatHB;  // fewest passes with L <= 10
  s.L = m - kLatHB * s.np < 8 ? 8 : m - kLatHB * s.np;
  int rest = m - s.L;
  for (int q = 0; q < s.np; q++) {  // 5 bits first, the remainder spread over the top passes
    const int w = (rest + (s.np - q) - 1) / (s.np - q);
    s.hb[q] = w;
    rest -= w;
  }
  return s;
}
static size_t lat_lds_bytes(int L, size_t cbytes) {
  return ((size_t)lds_stride(L) + (L ? (1u << (L - 1)) : 0)) * cbytes;
}

// the two top register passes as one tile pass: both 5 bits wide, the window
// of a block (2^(lo + 10) elements) below 2^30 bytes; its grid has as many
// blocks per vector as the top register pass (2^(lo - 3) = 2^(m - 13))
static bool lat_tile(const LatSched& s, size_t cbytes) {
  if (s.np < 2 || s.hb[s.np - 1] != 5 || s.hb[s.np - 2] != 5) return false;
  return (cbytes << (s.lo(s.np - 2) + 10)) <= ((size_t)1 << 30);
}

// blocks per vector of the last adjoint pass (the top register pass)
int lat_adj_blocks(int m, size_t /*cbytes*/) {
  const LatSched s = lat_sched(m);
  if (s.np == 0) return 1;
  return 1 << (m - s.hb[s.np - 1] - 8);
}

#define MTGP_LAT_KT(kt, MACRO, ...)                   \
  do {                                                \
    switch (kt) {                                     \
      case KT_SI1: MACRO(KT_SI1, __VA_ARGS__); break; \
      case KT_SI2: MACRO(KT_SI2, __VA_ARGS__); break; \
      default: MACRO(KT_SI3, __VA_ARGS__); break;     \
    }                                                 \
  } while (0)

// raw buffer addressing while the window of a block fits in 2^30 bytes
template <typename CR>
static bool lat_buf(int lo, int hb) {
  return ((int64_t)sizeof(cx<CR>) << (lo + hb)) <= ((int64_t)1 << 30);
}

template <typename CR, int SRC, int KT>
static void dif_reg(const LatTab& tab, int nvec, hipStream_t st, cx<CR>* work, int64_t vstride,
                    int m, int lo, int hb, const void* y, int y_f32, const uint32_t* gen,
                    const uint32_t* colshift, const Params* P, int d) {
  const dim3 grid(1u << (m - hb - 8), nvec);
  const bool buf = lat_buf<CR>(lo, hb);
#define MTGP_DIF_REG(HB, BUF)                                                                   \
  hipLaunchKernelGGL((lat_dif_reg_kernel<CR, CR, HB, SRC, KT, BUF>), grid, dim3(256), 0, st, tab, \
                     work, work, vstride, m, lo, y, y_f32, gen, colshift, P, d)
  if (hb == kLatHB) {
    if (buf) MTGP_DIF_REG(kLatHB, true);
    else MTGP_DIF_REG(kLatHB, false);
  } else {
    if (buf) MTGP_DIF_REG(4, true);
    else MTGP_DIF_REG(4, false);
  }
#undef MTGP_DIF_REG
}

// Forward transform of nvec vectors (columns when src == SRC_GEN, data when
// SRC_Y / SRC_X) of length 2^m into the bit-reversed spectrum, times scale;
// `work` holds the register passes (may alias spec when the types agree).
template <typename CR, typename SR>
int launch_lat_forward(int src, cx<CR>* work, cx<SR>* spec, int64_t vstride, int nvec, int m,
                       const void* y, int y_f32, double scale, const uint32_t* gen,
                       const uint32_t* colshift, const Params* P, const KDesc& kd,
                       hipStream_t st, int natural) {
  if (nvec <= 0) return 0;
  if (natural && !lat_natural_out(m)) return -1;
  const int kt = kt_of(kd.family, kd.order, kd.adaptive);
  const LatSched s = lat_sched(m);
  const LatTab tab = lat_tab();
  const bool tile = lat_tile(s, sizeof(cx<CR>));
  if (tile) {  // the two top passes in one
    const int lo = s.lo(s.np - 2);
    const dim3 gridT(1u << (m - 13), nvec);  // 2^(lo - 3) groups x 2^(m - lo - 10)
    const size_t lds = lat_tile_lds_bytes(sizeof(cx<CR>));
#define FT(KTV, SRCV)                                                                          \
  hipLaunchKernelGGL((lat_dif_tile_kernel<CR, SRCV, KTV>), gridT, dim3(256), lds, st, tab, work, \
                     vstride, m, lo, y, y_f32, gen, colshift, P, kd.d)
    if (src == SRC_GEN) MTGP_LAT_KT(kt, FT, SRC_GEN);
    else if (src == SRC_Y) FT(KT_SI1, SRC_Y);
    else FT(KT_SI1, SRC_X);
#undef FT
  }
  for (int q = tile ? s.np - 3 : s.np - 1; q >= 0; q--) {  // top pass first
    const int lo = s.lo(q), hb = s.hb[q];
    if (q == s.np - 1) {
#define FR(KTV, SRCV)                                                                          \
  dif_reg<CR, SRCV, KTV>(tab, nvec, st, work, vstride, m, lo, hb, y, y_f32, gen, colshift, P, \
                         kd.d)
      if (src == SRC_GEN) MTGP_LAT_KT(kt, FR, SRC_GEN);
      else if (src == SRC_Y) FR(KT_SI1, SRC_Y);
      else FR(KT_SI1, SRC_X);
#undef FR
    } else {
      dif_reg<CR, SRC_WORK, KT_SI1>(tab, nvec, st, work, vstride, m, lo, hb, y, y_f32, gen,
                                    colshift, P, kd.d);
    }
  }
  if (s.np > 0 && s.L <= 10) {  // multi-pass: the wave pass over the low bits
    if (natural)
      launch_dif_wave_natural<CR, SR>(s.L, nvec, st, work, spec, vstride, m, scale);
    else
      launch_dif_wave<CR, SR>(s.L, dim3(1u << (m - s.L - 2), nvec), st, work, spec, vstride,
                              scale);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  const dim3 grid2(1u << (m - s.L), nvec);
  const size_t lds = lat_lds_bytes(s.L, sizeof(cx<CR>));
#define FL(KTV, SRCV)                                                                          \
  hipLaunchKernelGGL((lat_dif_lds_kernel<CR, SR, SRCV, KTV>), grid2, dim3(256), lds, st, work, \
                     spec, vstride, m, s.L, scale, 0, y, y_f32, gen, colshift, P, kd.d)
  if (s.np > 0) FL(KT_SI1, SRC_WORK);
  else if (src == SRC_GEN) MTGP_LAT_KT(kt, FL, SRC_GEN);
  else if (src == SRC_Y) FL(KT_SI1, SRC_Y);
  else FL(KT_SI1, SRC_X);
#undef FL
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Adjoint: u = Re F omega, reduced against the regenerated column derivatives
// (partials: lat_adj_blocks(m) rows per vector, vector-major), or written
// (SINK_REAL, times scale) to real_out in natural order.  Overwrites work.
template <typename CR, typename SR>
int launch_lat_adjoint(int sink, const cx<SR>* spec, cx<CR>* work, double* real_out,
                       int64_t vstride, int nvec, int m, int conj_in, double scale,
                       const uint32_t* gen, const uint32_t* colshift, const Params* P,
                       const KDesc& kd, double* partials, hipStream_t st) {
  if (nvec <= 0) return 0;
  const int kt = kt_of(kd.family, kd.order, kd.adaptive);
  const LatSched s = lat_sched(m);
  const LatTab tab = lat_tab();
  const dim3 gridL(1u << (m - s.L), nvec);
  const size_t lds = lat_lds_bytes(s.L, sizeof(cx<CR>));
  const bool wave = s.np > 0 && s.L <= 10;  // multi-pass: the wave pass over the low bits
  if (wave) launch_dit_wave<CR, SR>(s.L, dim3(1u << (m - s.L - 2), nvec), st, spec, work, vstride,
                                    conj_in);
#define AL(DD, KTV, SINKV)                                                                    \
  hipLaunchKernelGGL((lat_dit_lds_kernel<CR, SR, SINKV, KTV, DD>), gridL, dim3(256), lds, st, \
                     spec, work, real_out, vstride, m, s.L, conj_in, scale, gen, colshift, P, \
                     kd.d, partials)
#define AL_D(DD, KTV) AL(DD, KTV, SINK_REDUCE)
  if (wave) {
  } else if (s.np > 0) {
    AL(2, KT_SI1, SINK_WORK);
  } else if (sink == SINK_REAL) {
    AL(2, KT_SI1, SINK_REAL);
  } else {
    switch (kt) {
      case KT_SI1: MTGP_DISPATCH_D(kd.d, AL_D, KT_SI1); break;
      case KT_SI2: MTGP_DISPATCH_D(kd.d, AL_D, KT_SI2); break;
      default: MTGP_DISPATCH_D(kd.d, AL_D, KT_SI3); break;
    }
  }
#undef AL_D
#undef AL
  // tile pass: with three or more register passes, the two lowest (work to
  // work; the reducing top pass keeps its register pass at 3 waves per SIMD),
  // with two, both of them with the final sink
  const bool low_tile = s.np >= 3 && s.hb[0] == 5 && s.hb[1] == 5 &&
                        (sizeof(cx<CR>) << (s.lo(0) + 10)) <= ((size_t)1 << 30);
  const bool top_tile = s.np == 2 && lat_tile(s, sizeof(cx<CR>));
  if (low_tile || top_tile) {
    const int lo = s.lo(0);
    const dim3 gridT(1u << (m - 13), nvec);  // 2^(lo - 3) groups x 2^(m - lo - 10)
    const size_t lds = lat_tile_lds_bytes(sizeof(cx<CR>));
#define AT(DD, KTV, SINKV)                                                                     \
  hipLaunchKernelGGL((lat_dit_tile_kernel<CR, SINKV, KTV, DD>), gridT, dim3(256), lds, st, tab, \
                     work, real_out, vstride, m, lo, scale, gen, colshift, P, kd.d, partials)
#define AT_D(DD, KTV) AT(DD, KTV, SINK_REDUCE)
    if (low_tile) {
      AT(2, KT_SI1, SINK_WORK);
    } else if (sink == SINK_REAL) {
      AT(2, KT_SI1, SINK_REAL);
    } else {
      switch (kt) {
        case KT_SI1: MTGP_DISPATCH_D(kd.d, AT_D, KT_SI1); break;
        case KT_SI2: MTGP_DISPATCH_D(kd.d, AT_D, KT_SI2); break;
        default: MTGP_DISPATCH_D(kd.d, AT_D, KT_SI3); break;
      }
    }
#undef AT_D
#undef AT
    if (top_tile) return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  for (int q = low_tile ? 2 : 0; q < s.np; q++) {
    const int lo = s.lo(q), hb = s.hb[q];
    const dim3 grid(1u << (m - hb - 8), nvec);
    const bool last = q == s.np - 1;
    const size_t stage = last && sink == SINK_REDUCE ? ((size_t)256 << hb) * sizeof(CR) : 0;
    const bool buf = lat_buf<CR>(lo, hb);
#define AR_HB(HB, DD, KTV, SINKV)                                                                \
  if (buf)                                                                                       \
    hipLaunchKernelGGL((lat_dit_reg_kernel<CR, HB, SINKV, KTV, DD, true>), grid, dim3(256),      \
                       stage, st, tab, work, real_out, vstride, m, lo, scale, gen, colshift, P,  \
                       kd.d, partials);                                                          \
  else                                                                                           \
    hipLaunchKernelGGL((lat_dit_reg_kernel<CR, HB, SINKV, KTV, DD, false>), grid, dim3(256),     \
                       stage, st, tab, work, real_out, vstride, m, lo, scale, gen, colshift, P,  \
                       kd.d, partials)
#define AR(DD, KTV, SINKV)                 \
  do {                                     \
    if (hb == kLatHB) {                    \
      AR_HB(kLatHB, DD, KTV, SINKV);       \
    } else {                               \
      AR_HB(4, DD, KTV, SINKV);            \
    }                                      \
  } while (0)
#define AR_D(DD, KTV) AR(DD, KTV, SINK_REDUCE)
    if (!last) {
      AR(2, KT_SI1, SINK_WORK);
    } else if (sink == SINK_REAL) {
      AR(2, KT_SI1, SINK_REAL);
    } else {
      switch (kt) {
        case KT_SI1: MTGP_DISPATCH_D(kd.d, AR_D, KT_SI1); break;
        case KT_SI2: MTGP_DISPATCH_D(kd.d, AR_D, KT_SI2); break;
        default: MTGP_DISPATCH_D(kd.d, AR_D, KT_SI3); break;
      }
    }
#undef AR_D
#undef AR
#undef AR_HB
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Standalone transform: 0 when one LDS pass covers 2^m (then the forward
// writes natural frequency order itself), else the forward needs a scratch
// spectrum that launch_lat_natural permutes.
int lat_single_pass(int m) { return lat_sched(m).np == 0; }

int lat_natural_out(int m) {
  const LatSched s = lat_sched(m);
  return s.np > 0 && s.L <= 10;
}

// one LDS pass straight into natural frequency order (m <= 12)
template <typename R>
int launch_lat_single_natural(int src, const void* x, int x_f32, cx<R>* X, int nvec, int m,
                              hipStream_t st) {
  if (nvec <= 0) return 0;
  const dim3 grid(1, nvec);
  const size_t lds = lat_lds_bytes(m, sizeof(cx<R>));
  const int64_t n = (int64_t)1 << m;
  if (src == SRC_Y)
    hipLaunchKernelGGL((lat_dif_lds_kernel<R, R, SRC_Y, KT_SI1>), grid, dim3(256), lds, st,
                       nullptr, X, n, m, m, 1.0, 1, x, x_f32, nullptr, nullptr, nullptr, 0);
  else
    hipLaunchKernelGGL((lat_dif_lds_kernel<R, R, SRC_X, KT_SI1>), grid, dim3(256), lds, st,
                       nullptr, X, n, m, m, 1.0, 1, x, x_f32, nullptr, nullptr, nullptr, 0);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// bit-reversed spectrum -> natural frequency order
template <typename R>
__global__ void lat_natural_kernel(const cx<R>* __restrict__ spec, cx<R>* __restrict__ X,
                                   int64_t nvec, int m) {
  const int64_t n = (int64_t)1 << m;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nvec * n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = q >> m, f = q & (n - 1);
    X[q] = spec[v * n + bitrev64(f, m)];
  }
}

// The same permutation through 32 x 32 LDS tiles (m >= 10): with f = a 2^(m-5)
// + b 2^5 + c (a, c of 5 bits), bitrev_m(f) = rev(c) 2^(m-5) + rev(b) 2^5 +
// rev(a), so the tile of one b reads 32 runs of 32 consecutive spectrum
// entries and writes 32 runs of 32 consecutive outputs.  Grid (2^(m-10), nvec).
template <typename R>
__global__ __launch_bounds__(256) void lat_natural_tiled_kernel(const cx<R>* __restrict__ spec,
                                                                cx<R>* __restrict__ X, int m) {
  __shared__ cx<R> t[32][33];
  const int64_t n = (int64_t)1 << m;
  const int64_t b = blockIdx.x;
  const int64_t rb = bitrev64(b, m - 10);
  const cx<R>* s = spec + (size_t)blockIdx.y * n;
  cx<R>* x = X + (size_t)blockIdx.y * n;
  for (int e = threadIdx.x; e < 1024; e += blockDim.x) {
    const int i = e >> 5, j = e & 31;
    t[i][j] = s[((int64_t)i << (m - 5)) | (rb << 5) | j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 1024; e += blockDim.x) {
    const int a = e >> 5, c = e & 31;
    x[((int64_t)a << (m - 5)) | (b << 5) | c] = t[bitrev64(c, 5)][bitrev64(a, 5)];
  }
}

int launch_lat_natural(const void* spec, int spec_f32, void* X, int64_t nvec, int m,
                       hipStream_t st) {
  if (nvec <= 0) return 0;
  if (m >= 10) {
    const dim3 grid(1u << (m - 10), (unsigned)nvec);
    if (spec_f32)
      hipLaunchKernelGGL(lat_natural_tiled_kernel<float>, grid, dim3(256), 0, st,
                         static_cast<const cx<float>*>(spec), static_cast<cx<float>*>(X), m);
    else
      hipLaunchKernelGGL(lat_natural_tiled_kernel<double>, grid, dim3(256), 0, st,
                         static_cast<const cx<double>*>(spec), static_cast<cx<double>*>(X), m);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  const int64_t total = nvec << m;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  if (spec_f32)
    hipLaunchKernelGGL(lat_natural_kernel<float>, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<const cx<float>*>(spec), static_cast<cx<float>*>(X), nvec, m);
  else
    hipLaunchKernelGGL(lat_natural_kernel<double>, dim3((unsigned)blocks), dim3(256), 0, st,
                       static_cast<const cx<double>*>(spec), static_cast<cx<double>*>(X), nvec, m);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template int launch_lat_single_natural<double>(int, const void*, int, cx<double>*, int, int,
                                               hipStream_t);
template int launch_lat_single_natural<float>(int, const void*, int, cx<float>*, int, int,
                                              hipStream_t);
template int launch_lat_forward<double, double>(int, cx<double>*, cx<double>*, int64_t, int, int,
                                                const void*, int, double, const uint32_t*,
                                                const uint32_t*, const Params*, const KDesc&,
                                                hipStream_t, int);
template int launch_lat_forward<double, float>(int, cx<double>*, cx<float>*, int64_t, int, int,
                                               const void*, int, double, const uint32_t*,
                                               const uint32_t*, const Params*, const KDesc&,
                                               hipStream_t, int);
template int launch_lat_forward<float, float>(int, cx<float>*, cx<float>*, int64_t, int, int,
                                              const void*, int, double, const uint32_t*,
                                              const uint32_t*, const Params*, const KDesc&,
                                              hipStream_t, int);
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

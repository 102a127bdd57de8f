// Transform passes over kernel columns and data vectors.
//
// A length-2^m Walsh-Hadamard transform (the V^dagger of Theorem "Fast GP
// computations" for digital sequences, unnormalised) is split by index bits:
//   pass A: bits [0, LB) of contiguous 2^LB blocks, LDS resident.  For kernel
//           columns the block is generated in registers first (fused column
//           evaluation, Eq. prod_kernel), so raw columns never reach HBM.
//   pass B: bits [lo, lo + hb); for hb <= 6 each thread holds the 2^hb
//           strided rows of one low index in registers (no LDS, rows
//           addressed through raw buffer resources); hb = 8, 10, 12 run in
//           one pass through registers and one LDS tile (fwht_hi_kernel);
//           other wider passes use tiles of KC consecutive low indices
//           times 2^hb strided rows, LDS resident.
// The stages of a Walsh-Hadamard transform commute, so the split needs no
// twiddles and the output stays in natural (Sylvester) order.
#include "colgen.h"

namespace mtgp {

// ---------------------------------------------------------------------------
// raw kernel columns (no transform): one thread per element
// ---------------------------------------------------------------------------
template <typename Real, int FAM, int ADAPT>
__global__ __launch_bounds__(256) void raw_cols_kernel(Real* __restrict__ base, int m, int ncols,
                                                       const uint32_t* __restrict__ gen,
                                                       const uint32_t* __restrict__ colshift,
                                                       const Params* __restrict__ P, KDesc kd) {
  const int64_t n = (int64_t)1 << m;
  const int64_t total = n * ncols;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int col = (int)(q >> m);
    const uint32_t i = (uint32_t)(q & (n - 1));
    const uint32_t* sh = colshift + (size_t)col * kd.d;
    Real c = RT<Real>::gamma(P);
    for (int j = 0; j < kd.d; j++) {
      const uint32_t u = FAM == FAM_DSEQ ? (dseq_z(gen + 32 * j, i) ^ sh[j])
                                         : (lat_z(gen[j], i, m) + sh[j]);
      c *= (Real)1 + RT<Real>::eta(P, j) * univ_value<Real, FAM, ADAPT>(kd.order, u, P);
    }
    base[q] = c;
  }
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
  if (LB == 12) {
    // 16 loads in flight per thread, bits 8 .. 11 in registers
    const int t = threadIdx.x;
    Real v[16];
#pragma unroll
    for (int k = 0; k < 16; k++) v[k] = p[t + 256 * k];
    reg_fwht<Real, 16>(v);
#pragma unroll
    for (int k = 0; k < 16; k++) lds[lds_at(0, stride, t + 256 * k)] = v[k];
    __syncthreads();
    lds_round<Real, 4>(lds, 1, LB, 0, stride);
    __syncthreads();
    lds_round<Real, 4>(lds, 1, LB, 4, stride);
    __syncthreads();
  } else {
    for (int i = threadIdx.x; i < nb; i += blockDim.x) lds[lds_at(0, stride, i)] = p[i];
    lds_fwht<Real>(lds, 1, LB, stride);
  }
  for (int i = threadIdx.x; i < nb; i += blockDim.x) p[i] = lds[lds_at(0, stride, i)];
}

// Pass B: butterflies over bits [lo, lo + hb) of vectors of length 2^m.
// Tile = KC consecutive low indices x 2^hb rows.  Tiles that share HBM lines
// (neighbouring low-index groups) get consecutive tile numbers, and the tile
// number is taken XCD-major (workgroups are dealt to the 8 XCDs round-robin),
// so those neighbours run at the same time on one XCD and share its L2.
// Arithmetic in TC; reads TIn, writes TOut (in place when in == out).
template <typename TC, typename TIn, typename TOut>
__global__ __launch_bounds__(256) void fwht_strided_kernel(const TIn* in, TOut* out,
                                                           int64_t vec_stride, int m, int lo,
                                                           int hb, int KC) {
  extern __shared__ __align__(16) unsigned char smem[];
  TC* lds = reinterpret_cast<TC*>(smem);
  const int nt = gridDim.x;
  int tile = blockIdx.x;
  if ((nt & 7) == 0) tile = (blockIdx.x & 7) * (nt >> 3) + (blockIdx.x >> 3);
  const int kc_bits = __ffs(KC) - 1;  // KC is a power of two
  const int tl_bits = lo - kc_bits;
  const int tl = tile & ((1 << tl_bits) - 1);
  const int ch = tile >> tl_bits;
  const int hi = lo + hb;
  const size_t off = (size_t)blockIdx.y * vec_stride + (size_t)tl * KC + ((size_t)ch << hi);
  const TIn* p = in + off;
  TOut* q_out = out + off;
  const int rows = 1 << hb;
  const int stride = lds_stride(hb);
  const int total = rows * KC;
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int kc = q & (KC - 1), r = q >> kc_bits;
    lds[lds_at(kc, stride, r)] = (TC)p[kc + ((size_t)r << lo)];
  }
  lds_fwht<TC>(lds, KC, hb, stride);
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int kc = q & (KC - 1), r = q >> kc_bits;
    q_out[kc + ((size_t)r << lo)] = (TOut)lds[lds_at(kc, stride, r)];
  }
}

// Pass B in registers (hb <= 6 bits, lo >= 8): thread = one low index of a
// group of 256 consecutive ones, holding its 2^HB strided rows.  Every row
// access of a wave is 64 consecutive elements, there is no LDS and no
// barrier, and each thread keeps 2^HB loads in flight.
template <typename TC, typename TIn, typename TOut, int HB>
__global__ __launch_bounds__(256) void fwht_reg_kernel(const TIn* in, TOut* out,
                                                       int64_t vec_stride, int lo) {
  constexpr int R = 1 << HB;
  const int64_t tile = blockIdx.x;
  const int gb = lo - 8;  // 256-index groups in the low part: 2^gb
  const int64_t grp = tile & (((int64_t)1 << gb) - 1);
  const int64_t hi = tile >> gb;
  const int64_t base = (int64_t)blockIdx.y * vec_stride + (hi << (lo + HB)) + (grp << 8) +
                       threadIdx.x;
  TC v[R];
#pragma unroll
  for (int r = 0; r < R; r++) v[r] = (TC)in[base + ((int64_t)r << lo)];
#pragma unroll
  for (int h = 1; h < R; h <<= 1) {
#pragma unroll
    for (int k = 0; k < R; k++) {
      if (!(k & h)) {
        const TC a = v[k], b = v[k + h];
        v[k] = a + b;
        v[k + h] = a - b;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; r++) out[base + ((int64_t)r << lo)] = (TOut)v[r];
}

// Raw buffer addressing (see buf_load): only the data stays in vector
// registers across the butterflies (a 64-bit address per row would double
// their count), so HB = 6 in double precision fits three waves per SIMD.
template <typename TC, typename TIn, typename TOut, int HB>
__global__ __launch_bounds__(256) void fwht_reg_buf_kernel(const TIn* in, TOut* out,
                                                           int64_t vec_stride, int lo) {
  constexpr int R = 1 << HB;
  const int64_t tile = blockIdx.x;
  const int gb = lo - 8;
  const int64_t grp = tile & (((int64_t)1 << gb) - 1);
  const int64_t hi = tile >> gb;
  const int64_t ub = (int64_t)blockIdx.y * vec_stride + (hi << (lo + HB)) + (grp << 8);
  const int nb_in = (int)(sizeof(TIn) << (lo + HB)), nb_out = (int)(sizeof(TOut) << (lo + HB));
  const __amdgpu_buffer_rsrc_t ri = buf_rsrc(in + ub, nb_in);
  const __amdgpu_buffer_rsrc_t ro = buf_rsrc(out + ub, nb_out);
  constexpr int HB1 = HB / 2, R1 = 1 << HB1, R2 = R >> HB1;
  TC v[R];
  // rows r = a * R1 + b: the transform over the bits of b for each a as the
  // rows arrive, then over the bits of a for each b, each group stored as
  // soon as it is done, so at most the R values of the thread are live
#pragma unroll
  for (int a = 0; a < R2; a++) {
#pragma unroll
    for (int b = 0; b < R1; b++) {
      const int r = a * R1 + b;
      v[r] = (TC)buf_load<TIn>(ri, threadIdx.x * (uint32_t)sizeof(TIn), ((uint32_t)r << lo) * sizeof(TIn));
    }
#pragma unroll
    for (int h = 1; h < R1; h <<= 1)
#pragma unroll
      for (int b = 0; b < R1; b++)
        if (!(b & h)) {
          const TC x = v[a * R1 + b], y = v[a * R1 + b + h];
          v[a * R1 + b] = x + y;
          v[a * R1 + b + h] = x - y;
        }
  }
#pragma unroll
  for (int b = 0; b < R1; b++) {
#pragma unroll
    for (int h = 1; h < R2; h <<= 1)
#pragma unroll
      for (int a = 0; a < R2; a++)
        if (!(a & h)) {
          const TC x = v[a * R1 + b], y = v[(a + h) * R1 + b];
          v[a * R1 + b] = x + y;
          v[(a + h) * R1 + b] = x - y;
        }
#pragma unroll
    for (int a = 0; a < R2; a++) {
      const int r = a * R1 + b;
      buf_store<TOut>((TOut)v[r], ro, threadIdx.x * (uint32_t)sizeof(TOut),
                      ((uint32_t)r << lo) * sizeof(TOut));
    }
  }
}

// Walsh-Hadamard transform of the 2^B register values of a thread: over the
// low B/2 index bits within each group of 2^(B/2), then over the high bits
// (group by group, so fewer temporaries are live than stage by stage).
template <typename TC, int B>
__device__ inline void reg_fwht_split(TC (&v)[1 << B]) {
  constexpr int B1 = B / 2, R1 = 1 << B1, R2 = (1 << B) >> B1;
#pragma unroll
  for (int a = 0; a < R2; a++)
#pragma unroll
    for (int h = 1; h < R1; h <<= 1)
#pragma unroll
      for (int b = 0; b < R1; b++)
        if (!(b & h)) {
          const TC x = v[a * R1 + b], y = v[a * R1 + b + h];
          v[a * R1 + b] = x + y;
          v[a * R1 + b + h] = x - y;
        }
#pragma unroll
  for (int b = 0; b < R1; b++)
#pragma unroll
    for (int h = 1; h < R2; h <<= 1)
#pragma unroll
      for (int a = 0; a < R2; a++)
        if (!(a & h)) {
          const TC x = v[a * R1 + b], y = v[(a + h) * R1 + b];
          v[a * R1 + b] = x + y;
          v[(a + h) * R1 + b] = x - y;
        }
}

// One pass over all H high bits [lo, lo + H), H in {8, 10, 12}: a block takes
// KC = 256 / 2^(H/2) adjacent low indices (a run of KC elements per row) over
// all 2^H rows hi = h1 + 2^(H/2) h2 of one vector.  Phase 1: thread (c, h1)
// holds the rows of every h2 in registers and transforms over h2 while its
// loads are in flight; phase 2 reads the rows of one h2 per thread back from
// an LDS tile and transforms over h1; phase 3 re-reads the tile in the
// phase-1 order, so the stores have the loads' pattern (rows 2^lo apart
// inside one 2^(lo + H/2) span).  Half the HBM traffic of two register
// passes, but the tile fills most of a CU's LDS (one block per CU, phases in
// sequence), so it does not always win; the schedule picks.  The blocks that
// share a 128-byte line sit on one XCD, next to each other in dispatch order
// (dispatch is round-robin over the 8 XCDs).
template <typename TC, typename TIn, typename TOut, int H>
__global__ __launch_bounds__(256) void fwht_hi_kernel(const TIn* in, TOut* out,
                                                      int64_t vec_stride, int lo) {
  constexpr int H1 = H / 2, R = 1 << H1, KB = 8 - H1, KC = 1 << KB;
  // LDS slot of (row hi, column c): one run of padding per 2^H1 rows puts the
  // 64 lanes of a phase-2 access on distinct banks
  constexpr int PAD = KC;
  extern __shared__ __align__(16) unsigned char smem[];
  TC* lds = reinterpret_cast<TC*>(smem);
  const int ncg = 1 << (lo - KB);  // column groups per vector
  int cg = blockIdx.x;
  if ((ncg & 31) == 0) {
    const int x = cg & 7, sl = cg >> 3;
    cg = ((sl >> 2) << 5) + (x << 2) + (sl & 3);
  }
  const int64_t vb = (int64_t)blockIdx.y * vec_stride + ((int64_t)cg << KB);
  const int c = threadIdx.x & (KC - 1), u = threadIdx.x >> KB;
  const __amdgpu_buffer_rsrc_t ri = buf_rsrc(in + vb, (int)(sizeof(TIn) << (lo + H)));
  const __amdgpu_buffer_rsrc_t ro = buf_rsrc(out + vb, (int)(sizeof(TOut) << (lo + H)));
  const uint32_t lane_in = ((uint32_t)c + ((uint32_t)u << lo)) * (uint32_t)sizeof(TIn);
  const uint32_t lane_out = ((uint32_t)c + ((uint32_t)u << lo)) * (uint32_t)sizeof(TOut);
  TC v[R];
  // phase 1: rows u + R k
#pragma unroll
  for (int k = 0; k < R; k++)
    v[k] = (TC)buf_load<TIn>(ri, lane_in, ((uint32_t)k << (lo + H1)) * (uint32_t)sizeof(TIn));
  reg_fwht_split<TC, H1>(v);
#pragma unroll
  for (int k = 0; k < R; k++) lds[(u + (k << H1)) * KC + c + k * PAD] = v[k];
  __syncthreads();
  // phase 2: rows q + R u (each thread reads and rewrites only its own slots)
#pragma unroll
  for (int q = 0; q < R; q++) v[q] = lds[(q + (u << H1)) * KC + c + u * PAD];
  reg_fwht_split<TC, H1>(v);
#pragma unroll
  for (int q = 0; q < R; q++) lds[(q + (u << H1)) * KC + c + u * PAD] = v[q];
  __syncthreads();
  // phase 3: rows u + R k again
#pragma unroll
  for (int k = 0; k < R; k++)
    buf_store<TOut>((TOut)lds[(u + (k << H1)) * KC + c + k * PAD], ro, lane_out,
                    ((uint32_t)k << (lo + H1)) * (uint32_t)sizeof(TOut));
}

// One pass over the 12 high bits [lo, lo + 12) with a quarter-size LDS
// exchange.  A block takes KC (2, 4 or 8) adjacent low indices c over all
// 4096 rows h = a + 64 b of one vector; thread (c, u), group g = u / 16 (a
// wave or two for KC >= 4).  The rows stay in registers (64 per thread); the
// LDS only carries one quarter of the transpose at a time, KC x 64 x 16
// values.
//
// Phase 1: the thread holds rows a = u, b = 0 .. 63 and transforms over b.
// Its input block q (b in [16q, 16q + 16)) is negated when popcount(q & g)
// is odd, which by the XOR-shift rule of the Walsh transform,
//   sum_s (-1)^{k.s} (-1)^{t.s} x[s] = X[k ^ t],   t = 16 g,
// leaves frequency b = k ^ 16 g in register slot k: slot block q holds b
// block q ^ g.  Exchange, rounds r = 0 .. 3: every thread writes its slot
// block r (b block r ^ g, so the rows b = 16 (r ^ g) + i of a = u) to a
// 64 x 16 LDS grid per column, and reads back into the same slots the 16
// values (a = 16 (r ^ g) + j, b = u); the slot indices stay compile-time and
// each round moves a quarter of the tile.  Phase 2: slot s now holds
// a = s ^ 16 g, so the transform over the slots gives
//   (-1)^{popcount((k >> 4) & g)} Y[k]
// in slot k, the same per-block sign as phase 1's input, undone before the
// stores of rows k + 64 u.  Runs of adjacent column groups (about 1 KiB of
// each row) sit on one XCD, next to each other in dispatch order (dispatch is
// round-robin over the 8 XCDs), so each row's span reaches the memory
// channels together.
constexpr int HI12_AS = 17, HI12_CS = 64 * HI12_AS + 8;

// LDS bytes of fwht_hi12_kernel with KC columns per block
static size_t hi12_lds_bytes(int KC, size_t tc_bytes) { return (size_t)KC * HI12_CS * tc_bytes; }

// multiplies register block q by (-1)^popcount(q & g) (exact)
template <typename TC>
__device__ inline void negate_blocks(TC (&v)[64], int g) {
#pragma unroll
  for (int q = 1; q < 4; q++) {
    const TC sg = (__builtin_popcount(q & g) & 1) ? (TC)-1 : (TC)1;
#pragma unroll
    for (int i = 0; i < 16; i++) v[16 * q + i] *= sg;
  }
}

// Layouts of a vector: natural (row h of column group cg at cg KC + c + 2^lo h)
// or, for the output with KC = 8, in runs (groups of 16 low indices, each
// group's 4096 rows x 16 values contiguous: run_index; the block writes its
// 8-column half of every row) with the halves of the row index swapped (row
// k + 64 u stored at u + 64 k), so a wave store covers 8 consecutive rows of
// the run, 64 bytes each, and the neighbouring block on the same XCD fills
// the other half of each 128-byte line.
template <typename TC, typename TIn, typename TOut, int KC>
__global__ __launch_bounds__(64 * KC) void fwht_hi12_kernel(const TIn* in, TOut* out,
                                                            int64_t vec_stride, int lo, int xg,
                                                            int out_run) {
  constexpr int KB = KC == 8 ? 3 : KC == 4 ? 2 : 1, AS = HI12_AS, CS = HI12_CS;
  extern __shared__ __align__(16) unsigned char smem[];
  TC* X = reinterpret_cast<TC*>(smem);
  const int ncg = 1 << (lo - KB);
  int cg = blockIdx.x;
  // XCD x takes runs of 2^xg adjacent column groups (xg < 0: dispatch order)
  if (xg >= 0) {
    const int x = cg & 7, sl = cg >> 3;
    cg = ((sl >> xg) << (xg + 3)) + (x << xg) + (sl & ((1 << xg) - 1));
  }
  const int64_t vcol = (int64_t)blockIdx.y * vec_stride;
  const int64_t vnat = vcol + ((int64_t)cg << KB);
  const int64_t vrun = vcol + ((int64_t)(cg >> 1) << 16) + ((cg & 1) << 3);
  const int c = threadIdx.x & (KC - 1), u = threadIdx.x >> KB;
  // the group u / 16 is wave-uniform for KC >= 4
  int g = u >> 4;
  if constexpr (KC >= 4) g = __builtin_amdgcn_readfirstlane(g);
  const __amdgpu_buffer_rsrc_t ri = buf_rsrc(in + vnat, (int)(sizeof(TIn) << (lo + 12)));
  const __amdgpu_buffer_rsrc_t ro =
      out_run ? buf_rsrc(out + vrun, (int)(sizeof(TOut) << 16))
              : buf_rsrc(out + vnat, (int)(sizeof(TOut) << (lo + 12)));
  // row h = u + 64 b at c + 2^lo u + 2^(lo+6) b
  const uint32_t lane_in = ((uint32_t)c + ((uint32_t)u << lo)) * (uint32_t)sizeof(TIn);
  TC v[64];
#pragma unroll
  for (int b = 0; b < 64; b++)
    v[b] = (TC)buf_load<TIn>(ri, lane_in, ((uint32_t)b << (lo + 6)) * (uint32_t)sizeof(TIn));
  // all 64 loads in flight before the first butterfly
  __builtin_amdgcn_sched_barrier(0);
  negate_blocks<TC>(v, g);
  reg_fwht_split<TC, 6>(v);
  TC* Xc = X + c * CS;
#pragma unroll
  for (int r = 0; r < 4; r++) {
#pragma unroll
    for (int i = 0; i < 16; i++) Xc[u * AS + i] = v[16 * r + i];
    __syncthreads();
    const TC* src = Xc + (((r ^ g) << 4) * AS) + (u & 15);
#pragma unroll
    for (int j = 0; j < 16; j++) v[16 * r + j] = src[j * AS];
    if (r < 3) __syncthreads();
  }
  reg_fwht_split<TC, 6>(v);
  negate_blocks<TC>(v, g);
  // row k + 64 u: natural c + 2^(lo+6) u + 2^lo k, in runs (halves swapped)
  // c + 16 u + 1024 k
  const uint32_t lane_out =
      ((uint32_t)c + ((uint32_t)u << (out_run ? 4 : lo + 6))) * (uint32_t)sizeof(TOut);
  const int sh_out = out_run ? 10 : lo;
#pragma unroll
  for (int k = 0; k < 64; k++)
    buf_store<TOut>((TOut)v[k], ro, lane_out, ((uint32_t)k << sh_out) * (uint32_t)sizeof(TOut));
}

static size_t fwht_hi_lds_bytes(int H, size_t tc_bytes) {
  const int R = 1 << (H / 2), KC = 256 / R;
  return ((size_t)KC << H) * tc_bytes + (size_t)R * KC * tc_bytes;
}

// one pass over the hb high bits when hb is 8, 10 or 12, the KC columns of a
// block fit in the low part and a block's window stays below 2^30 bytes
static bool fwht_hi_ok(int lo, int hb, size_t in_bytes, size_t out_bytes) {
  if (hb != 8 && hb != 10 && hb != 12) return false;
  const int KB = hb == 12 ? 3 : 8 - hb / 2;  // (12 bits: up to 8 columns per block)
  const size_t w = (in_bytes > out_bytes ? in_bytes : out_bytes) << (lo + hb);
  return lo >= KB && w <= ((size_t)1 << 30);
}

// 12 bits: the widest column group (2, 4 or 8 columns) whose exchange grid
// fits the schedule's tile budget
static int hi12_kc(size_t tile, size_t tc_bytes) {
  return hi12_lds_bytes(8, tc_bytes) <= tile ? 8 : hi12_lds_bytes(4, tc_bytes) <= tile ? 4 : 2;
}

template <typename TC, typename TIn, typename TOut>
void launch_hi_pass(const TIn* in, TOut* out, int64_t vec_stride, int nv, int lo, int hb,
                    size_t tile, int out_run, hipStream_t st) {
  const dim3 grid(1u << (lo - (8 - hb / 2)), (unsigned)nv);
  const size_t lds = fwht_hi_lds_bytes(hb, sizeof(TC));
  if (hb == 12) {
    const int kc = hi12_kc(tile, sizeof(TC));
    const size_t l12 = hi12_lds_bytes(kc, sizeof(TC));
    const int kb = kc == 8 ? 3 : kc == 4 ? 2 : 1;
    const dim3 g12(1u << (lo - kb), (unsigned)nv);
    // XCD placement: runs of about 1 KiB of input per row on each XCD (measured
    // at 2^24-point columns: 512 B runs 1.99 ms, 1 KiB 1.70 ms per forward
    // pass), at most an eighth of the column groups each
    int xg = 0;
    while (((size_t)kc * sizeof(TIn) << (xg + 1)) <= 1024) xg++;
    const int ncg_bits = lo - kb;
    if (xg > ncg_bits - 3) xg = ncg_bits - 3;
    if (kc == 8)
      hipLaunchKernelGGL((fwht_hi12_kernel<TC, TIn, TOut, 8>), g12, dim3(512), l12, st, in, out,
                         vec_stride, lo, xg, out_run);
    else if (kc == 4)
      hipLaunchKernelGGL((fwht_hi12_kernel<TC, TIn, TOut, 4>), g12, dim3(256), l12, st, in, out,
                         vec_stride, lo, xg, 0);
    else
      hipLaunchKernelGGL((fwht_hi12_kernel<TC, TIn, TOut, 2>), g12, dim3(128), l12, st, in, out,
                         vec_stride, lo, xg, 0);
  } else if (hb == 10)
    hipLaunchKernelGGL((fwht_hi_kernel<TC, TIn, TOut, 10>), grid, dim3(256), lds, st, in, out,
                       vec_stride, lo);
  else
    hipLaunchKernelGGL((fwht_hi_kernel<TC, TIn, TOut, 8>), grid, dim3(256), lds, st, in, out,
                       vec_stride, lo);
}

template <typename TC, typename TIn, typename TOut>
void launch_reg_pass(const TIn* in, TOut* out, int64_t vec_stride, int nv, int m, int lo, int hb,
                     hipStream_t st) {
  const dim3 grid((unsigned)((int64_t)1 << (m - hb - 8)), (unsigned)nv);
  // buffer addressing needs the window of a block (2^(lo+hb) elements of the
  // wider type) below 2^31 bytes
  const bool buf = lo + hb + 3 <= 30;
  switch (hb) {
#define MTGP_REGP(H)                                                                              \
  case H:                                                                                         \
    if (buf)                                                                                      \
      hipLaunchKernelGGL((fwht_reg_buf_kernel<TC, TIn, TOut, H>), grid, dim3(256), 0, st, in,    \
                         out, vec_stride, lo);                                                    \
    else                                                                                          \
      hipLaunchKernelGGL((fwht_reg_kernel<TC, TIn, TOut, H>), grid, dim3(256), 0, st, in, out,   \
                         vec_stride, lo);                                                         \
    break;
    MTGP_REGP(1)
    MTGP_REGP(2)
    MTGP_REGP(3)
    MTGP_REGP(4)
    MTGP_REGP(5)
    MTGP_REGP(6)
#undef MTGP_REGP
    default: break;
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
size_t gen_cols_lds_bytes(int LB, int real_bytes) { return (size_t)lds_stride(LB) * real_bytes; }

// Passes over bits [lb(m), m) in TC arithmetic.  The first pass reads `first`
// (TIn), the last writes `last` (TOut); intermediate results live in `work`
// (TC).  Any of them may alias when the types agree.
// bits of the next strided pass from bit lo of a length-2^m transform
static int next_pass_bits(const Sched& sc, int lo, int m, size_t in_bytes, size_t out_bytes) {
  const int r = m - lo;
  if (sc.b_bits > 0) return r < sc.b_bits ? r : sc.b_bits;
  // by size: the whole remainder in one pass where a one-pass kernel takes it
  return r <= 12 && fwht_hi_ok(lo, r, in_bytes, out_bytes) ? r : (r < 6 ? r : 6);
}

bool strided_runs(const Sched& sc, int m, size_t tc_bytes, size_t in_bytes, size_t out_bytes) {
  const int lo = sc.lb(m);
  const size_t ib = tc_bytes > in_bytes ? tc_bytes : in_bytes;
  const size_t ob = tc_bytes > out_bytes ? tc_bytes : out_bytes;
  return m - lo == 12 && lo >= 4 && next_pass_bits(sc, lo, m, ib, ob) == 12 &&
         fwht_hi_ok(lo, 12, ib, ob) && hi12_kc(sc.b_tile, tc_bytes) == 8;
}

template <typename TC, typename TIn, typename TOut>
int launch_strided(const TIn* first, TC* work, TOut* last, int64_t vec_stride, int64_t nvec,
                   int m, const Sched& sc, hipStream_t st, int runs) {
  if (runs && !strided_runs(sc, m, sizeof(TC), sizeof(TIn), sizeof(TOut))) return -1;
  int lo = sc.lb(m);
  bool is_first = true;
  while (lo < m) {
    const int hb = next_pass_bits(sc, lo, m,
                                  sizeof(TC) > sizeof(TIn) ? sizeof(TC) : sizeof(TIn),
                                  sizeof(TC) > sizeof(TOut) ? sizeof(TC) : sizeof(TOut));
    const bool is_last = lo + hb >= m;
    if (fwht_hi_ok(lo, hb, sizeof(TC) > sizeof(TIn) ? sizeof(TC) : sizeof(TIn),
                   sizeof(TC) > sizeof(TOut) ? sizeof(TC) : sizeof(TOut))) {
      for (int64_t v0 = 0; v0 < nvec; v0 += 65535) {
        const int nv = (int)((nvec - v0) < 65535 ? (nvec - v0) : 65535);
        const int64_t o = v0 * vec_stride;
        if (is_first && is_last)
          launch_hi_pass<TC, TIn, TOut>(first + o, last + o, vec_stride, nv, lo, hb, sc.b_tile,
                                        runs, st);
        else if (is_first)
          launch_hi_pass<TC, TIn, TC>(first + o, work + o, vec_stride, nv, lo, hb, sc.b_tile, 0,
                                     st);
        else if (is_last)
          launch_hi_pass<TC, TC, TOut>(work + o, last + o, vec_stride, nv, lo, hb, sc.b_tile, 0,
                                       st);
        else
          launch_hi_pass<TC, TC, TC>(work + o, work + o, vec_stride, nv, lo, hb, sc.b_tile, 0,
                                     st);
      }
      is_first = false;
      lo += hb;
      continue;
    }
    if (hb <= 6 && lo >= 8) {
      for (int64_t v0 = 0; v0 < nvec; v0 += 65535) {
        const int nv = (int)((nvec - v0) < 65535 ? (nvec - v0) : 65535);
        const int64_t o = v0 * vec_stride;
        if (is_first && is_last)
          launch_reg_pass<TC, TIn, TOut>(first + o, last + o, vec_stride, nv, m, lo, hb, st);
        else if (is_first)
          launch_reg_pass<TC, TIn, TC>(first + o, work + o, vec_stride, nv, m, lo, hb, st);
        else if (is_last)
          launch_reg_pass<TC, TC, TOut>(work + o, last + o, vec_stride, nv, m, lo, hb, st);
        else
          launch_reg_pass<TC, TC, TC>(work + o, work + o, vec_stride, nv, m, lo, hb, st);
      }
      is_first = false;
      lo += hb;
      continue;
    }
    int KC = 1;  // largest power of two with KC padded sequences inside the tile budget
    while ((size_t)(2 * KC) * lds_stride(hb) * sizeof(TC) <= sc.b_tile && 2 * KC <= (1 << lo))
      KC *= 2;
    const int64_t tiles = ((int64_t)1 << lo) / KC * ((int64_t)1 << (m - lo - hb));
    const size_t lds = (size_t)KC * lds_stride(hb) * sizeof(TC);
    for (int64_t v0 = 0; v0 < nvec; v0 += 65535) {
      const int64_t nv = (nvec - v0) < 65535 ? (nvec - v0) : 65535;
      const dim3 grid((unsigned)tiles, (unsigned)nv);
      const int64_t o = v0 * vec_stride;
      if (is_first && is_last)
        hipLaunchKernelGGL((fwht_strided_kernel<TC, TIn, TOut>), grid, dim3(256), lds, st,
                           first + o, last + o, vec_stride, m, lo, hb, KC);
      else if (is_first)
        hipLaunchKernelGGL((fwht_strided_kernel<TC, TIn, TC>), grid, dim3(256), lds, st,
                           first + o, work + o, vec_stride, m, lo, hb, KC);
      else if (is_last)
        hipLaunchKernelGGL((fwht_strided_kernel<TC, TC, TOut>), grid, dim3(256), lds, st,
                           work + o, last + o, vec_stride, m, lo, hb, KC);
      else
        hipLaunchKernelGGL((fwht_strided_kernel<TC, TC, TC>), grid, dim3(256), lds, st, work + o,
                           work + o, vec_stride, m, lo, hb, KC);
    }
    is_first = false;
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
  if (hipGetLastError() != hipSuccess) return -1;
  return launch_strided<Real, Real, Real>(base, base, base, vec_stride, nvec, m, sc, st);
}

template <typename Real, typename TOut>
int launch_gen_fwd(TOut* base, int64_t col_stride, int ncols, int m, const uint32_t* gen,
                   const uint32_t* colshift, const Params* P, const KDesc& kd, const Sched& sc,
                   hipStream_t st) {
  if (ncols <= 0) return 0;
  switch (kt_of(kd.family, kd.order, kd.adaptive)) {
    case KT_DSI1:
      return launch_gen_fwd_kt<Real, TOut, KT_DSI1>(base, col_stride, ncols, m, gen, colshift, P,
                                                    kd.d, sc, st);
    case KT_DSI2:
      return launch_gen_fwd_kt<Real, TOut, KT_DSI2>(base, col_stride, ncols, m, gen, colshift, P,
                                                    kd.d, sc, st);
    case KT_DSI3:
      return launch_gen_fwd_kt<Real, TOut, KT_DSI3>(base, col_stride, ncols, m, gen, colshift, P,
                                                    kd.d, sc, st);
    case KT_DSI4:
      return launch_gen_fwd_kt<Real, TOut, KT_DSI4>(base, col_stride, ncols, m, gen, colshift, P,
                                                    kd.d, sc, st);
    case KT_DSIA:
      return launch_gen_fwd_kt<Real, TOut, KT_DSIA>(base, col_stride, ncols, m, gen, colshift, P,
                                                    kd.d, sc, st);
    default: return -1;
  }
}

template <typename Real>
int launch_raw_cols(Real* base, int ncols, int m, const uint32_t* gen, const uint32_t* colshift,
                    const Params* P, const KDesc& kd, hipStream_t st) {
  if (ncols <= 0) return 0;
  const int64_t total = ((int64_t)1 << m) * ncols;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65535) blocks = 65535;
  const dim3 grid((unsigned)blocks);
  if (kd.family == FAM_DSEQ) {
    if (kd.adaptive)
      hipLaunchKernelGGL((raw_cols_kernel<Real, FAM_DSEQ, 1>), grid, dim3(256), 0, st, base, m,
                         ncols, gen, colshift, P, kd);
    else
      hipLaunchKernelGGL((raw_cols_kernel<Real, FAM_DSEQ, 0>), grid, dim3(256), 0, st, base, m,
                         ncols, gen, colshift, P, kd);
  } else {
    hipLaunchKernelGGL((raw_cols_kernel<Real, FAM_LAT, 0>), grid, dim3(256), 0, st, base, m, ncols,
                       gen, colshift, P, kd);
  }
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
template int launch_strided<double, double, double>(const double*, double*, double*, int64_t,
                                                    int64_t, int, const Sched&, hipStream_t, int);
template int launch_strided<double, double, float>(const double*, double*, float*, int64_t,
                                                   int64_t, int, const Sched&, hipStream_t, int);
template int launch_strided<double, float, double>(const float*, double*, double*, int64_t,
                                                   int64_t, int, const Sched&, hipStream_t, int);
template int launch_strided<float, float, float>(const float*, float*, float*, int64_t, int64_t,
                                                 int, const Sched&, hipStream_t, int);
template int launch_gen_fwd<double, double>(double*, int64_t, int, int, const uint32_t*,
                                            const uint32_t*, const Params*, const KDesc&,
                                            const Sched&, hipStream_t);
template int launch_gen_fwd<double, float>(float*, int64_t, int, int, const uint32_t*,
                                           const uint32_t*, const Params*, const KDesc&,
                                           const Sched&, hipStream_t);
template int launch_gen_fwd<float, float>(float*, int64_t, int, int, const uint32_t*,
                                          const uint32_t*, const Params*, const KDesc&,
                                          const Sched&, hipStream_t);
template int launch_raw_cols<double>(double*, int, int, const uint32_t*, const uint32_t*,
                                     const Params*, const KDesc&, hipStream_t);
template int launch_raw_cols<float>(float*, int, int, const uint32_t*, const uint32_t*,
                                    const Params*, const KDesc&, hipStream_t);
template int launch_scale<double>(double*, int64_t, double, hipStream_t);
template int launch_scale<float>(float*, int64_t, float, hipStream_t);

}  // namespace mtgp

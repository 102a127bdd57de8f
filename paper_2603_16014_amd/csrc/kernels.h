// Internal declarations shared by the HIP translation units of the library.
#pragma once
#include "common.h"

namespace mtgp {

// Pass A covers index bits [0, PASS_A_MAX_BITS); 256 threads hold up to
// MAXE = 2^13 / 256 elements each.  Pass B covers <= PASS_B_MAX_BITS more bits
// per launch with a tile of about PASS_B_TILE_BYTES of LDS.
constexpr int PASS_A_MAX_BITS = 13;
constexpr int MAXE = (1 << PASS_A_MAX_BITS) / 256;
constexpr int PASS_B_MAX_BITS = 11;
constexpr size_t PASS_B_TILE_BYTES = 73728;

// Lattice digit of natural-order index j: (j g mod 2^m) 2^(32-m), i.e. the
// point j g / n mod 1 of the unshifted rank-1 lattice with n = 2^m.
__device__ inline uint32_t lat_z(uint32_t g, uint32_t j, int m) {
  return (uint32_t)((uint64_t)(j * g) << (32 - m));
}

// Univariate kernel value; the adaptive DSI kernel weights Khat_1..4 by b.
template <typename Real, int FAM, int ADAPT>
__device__ inline Real univ_value(int order, uint32_t u, const Params* __restrict__ P) {
  if (ADAPT) {
    Real k[4];
    dsi_khat_all<Real>(u, k);
    return RT<Real>::bw(P, 0) * k[0] + RT<Real>::bw(P, 1) * k[1] + RT<Real>::bw(P, 2) * k[2] +
           RT<Real>::bw(P, 3) * k[3];
  }
  return univ<Real, FAM>(order, u);
}

// Task-pair -> column index map, and per-column scale / multiplicity.
// Entry i of a 4-byte-aligned uint8 row, taken from its dword: kernel
// arguments are read by dword scalar loads, while a byte read is a vector
// load that the address arithmetic using it has to wait for, one at a time.
// Column indices reach MTGP_MAXCOL - 1 = 135, so the entries are unsigned
// and read back zero-extended.
__host__ __device__ inline int u8_at(const uint8_t* row, int i) {
  uint32_t w;
  __builtin_memcpy(&w, row + (i & ~3), 4);
  return (int)((w >> (8 * (i & 3))) & 0xffu);
}

struct alignas(4) PairMap {
  uint8_t col[MTGP_MAXT][MTGP_MAXT];
  __host__ __device__ inline int at(int j, int i) const { return u8_at(col[j], i); }
};

// Transform schedule: pass A covers a_bits low index bits, each pass B at
// most b_bits more, with an LDS tile of about b_tile bytes.
struct Sched {
  int a_bits = 12;
  // bits per strided pass; 0: by size (one pass over a remainder of 8, 10
  // or 12 bits, else register passes of at most 6 bits)
  int b_bits = 0;
  size_t b_tile = 73728;
  // workgroups per CU of the fused generation / reduction kernels (0: as
  // many as fit), capped through their LDS request so that the strided
  // passes overlapped with them find room on every CU
  int fused_cap = 0;
  int lb(int m) const { return m < a_bits ? m : a_bits; }
  size_t fused_lds(size_t need) const {
    if (fused_cap <= 0) return need;
    const size_t cap = ((size_t)160 * 1024) / (size_t)(fused_cap + 1) + 1024;
    return need > cap ? need : cap;
  }
};

// Gray-code step table of the digital-sequence fused kernels, stored after
// the d x 32 generating columns: row k < GRAY_ROWS holds, per dimension j,
// z_j(256 gray(k)) with gray(k) = k ^ (k >> 1) (GRAY_STRIDE words per row).
constexpr int GRAY_ROWS = 32, GRAY_STRIDE = 32;
__host__ __device__ inline const uint32_t* gray_table(const uint32_t* gen, int d) {
  return gen + 32 * d;
}

// Digital-net adjoint reduction: one workgroup reduces adj_group(nb)
// consecutive low-bit blocks of a column (of nb), so a column writes
// nb / adj_group(nb) rows of the adjoint partial table.  More blocks per
// workgroup spread the per-thread digit set-up over more elements (2^24-point
// columns, 2^12-point blocks: 4 -> 8 blocks took the reduction from 2.13 to
// 2.11 ms mixed, 2.20 to 2.14 ms FP64).
inline int adj_group(int64_t nb) { return nb >= 8 ? 8 : (int)nb; }
// Digital-net column generation: consecutive low-bit blocks per workgroup
// (2 -> 4 at the same size: 1.65 -> 1.57 ms).
inline int gen_group(int64_t nb) { return nb >= 4 ? 4 : (int)nb; }
inline int64_t dseq_adj_rows(int m, int lb) {
  const int64_t nb = (int64_t)1 << (m - lb);
  return nb / adj_group(nb);
}

// ---- transform.hip
size_t gen_cols_lds_bytes(int LB, int real_bytes);
template <typename Real>
int launch_fwht(Real* base, int64_t vec_stride, int64_t nvec, int m, const Sched& sc,
                hipStream_t st);
// passes over bits [lb(m), m): first pass reads `first`, last writes `last`,
// intermediates in `work` (arithmetic in TC).  runs != 0 (only where
// strided_runs holds): `last` is written in the run layout with the halves
// of the row index swapped.
template <typename TC, typename TIn, typename TOut>
int launch_strided(const TIn* first, TC* work, TOut* last, int64_t vec_stride, int64_t nvec,
                   int m, const Sched& sc, hipStream_t st, int runs = 0);
// Whether the strided passes of a length-2^m transform are one 12-bit pass
// with 8 columns per block, which can write the run layout: the 2^lb low
// indices in groups of 16, each group's 4096 rows x 16 values contiguous
// (run_index), so a row of a group is one 128-byte line in FP64.
bool strided_runs(const Sched& sc, int m, size_t tc_bytes, size_t in_bytes, size_t out_bytes);
__host__ __device__ inline int64_t run_index(int h, int l) {
  return ((int64_t)(l >> 4) << 16) + ((int64_t)h << 4) + (l & 15);
}
// the row of block h in the run layout written by the adjoint's one pass
__host__ __device__ inline int run_swap(int h) { return ((h & 63) << 6) | (h >> 6); }
// kernel columns generated and transformed over the low index bits
template <typename Real, typename TOut>
int launch_gen_fwd(TOut* base, int64_t col_stride, int ncols, int m, const uint32_t* gen,
                   const uint32_t* colshift, const Params* P, const KDesc& kd, const Sched& sc,
                   hipStream_t st);
// per kernel type (fused_eval.h; instantiated in fused_*.hip)
template <typename Real, typename TOut, int KT>
int launch_gen_fwd_kt(TOut* base, int64_t col_stride, int ncols, int m, const uint32_t* gen,
                      const uint32_t* colshift, const Params* P, int d, const Sched& sc,
                      hipStream_t st);
template <typename Real, typename TIn, int KT>
int launch_adj_reduce_kt(const TIn* base, int64_t col_stride, int ncols, int m,
                         const uint32_t* gen, const uint32_t* colshift, const Params* P, int d,
                         double* partials, const Sched& sc, hipStream_t st, int run);
template <typename Real>
int launch_raw_cols(Real* base, int ncols, int m, const uint32_t* gen, const uint32_t* colshift,
                    const Params* P, const KDesc& kd, hipStream_t st);
template <typename Real>
int launch_scale(Real* x, int64_t n, Real s, hipStream_t st);

// ---- adjoint.hip
// Number of FP64 partial sums written per block by the derivative reduction.
__host__ __device__ inline int adj_nq(int d) { return d + 5; }
// run: the weights are in the run layout with swapped rows (strided_runs)
template <typename Real, typename TIn>
int launch_adj_reduce(const TIn* base, int64_t col_stride, int ncols, int m, const uint32_t* gen,
                      const uint32_t* colshift, const Params* P, const KDesc& kd, double* partials,
                      const Sched& sc, hipStream_t st, int run = 0);

// ---- solve.hip
int launch_clear_status(int* status, hipStream_t st);
int launch_prep(const double* theta, Params* P, const KDesc& kd, int* status, hipStream_t st);
// T padded to the factorisation template size, and the number of FP64
// partial sums per block of the solves (equal sizes and the elimination):
//   [0] quad, [1] log det, [2 + t] G_tt = sum_f W_tt lambda_tt,
//   [2 + TM + t] sum_f W_tt, [2 + 2 TM + t] ahat_t(0).
// The cross-task sums G_tu (t != u) are not formed here: the adjoint weights
// of a pair column are written without their R_tu factor, so the adjoint
// reduction's sum of w c over that column is 2 G_tu, and R_tu is applied to
// the column's derivative sums in the chain rule.
__host__ __device__ inline int solve_tm(int T) { return T <= 1 ? 1 : T <= 2 ? 2 : T <= 4 ? 4 : T <= 8 ? 8 : 16; }
__host__ __device__ inline int solve_ns(int T) { return 2 + 3 * solve_tm(T); }
// blocks of the equal-size solves (grid-stride over frequencies beyond)
inline int64_t solve_blocks(int64_t n) { return (n + 255) / 256; }
template <typename Real>
// yhat: the data transform at the spectrum's storage precision; yhat0: the
// FP64 transform, of which the solves read frequency 0 only
int launch_solve_eq(Real* cols, int64_t n, const PairMap& pm, int ncol, const Real* yhat,
                    const double* yhat0, const Params* P, const KDesc& kd, bool grad,
                    double* partials, double* ahat, int* status, hipStream_t st);
int launch_narrow(const double* in, float* out, int64_t n, hipStream_t st);
constexpr int COLSUM_BLOCKS = 256;
int launch_colsum(const double* in, int64_t nrows, int ncols, double* out, int nblk,
                  hipStream_t st);
template <typename SR>
int launch_solve_eq_c(SR* cols, int64_t n, const PairMap& pm, const SR* yhat, const double* yhat0,
                      const Params* P, const KDesc& kd, bool grad, double* partials, double* ahat,
                      int* status, hipStream_t st);
// Kernel column c: the task pair (t, u) it serves (t == u: a diagonal column,
// whose weights already carry R) and its rows in the adjoint partial table.
struct ColInfo {
  int32_t t, u;
  int64_t row_off, row_cnt;
};
// per-column sums of the adjoint partial table: out[c][nq]
int launch_colseg(const double* in, const ColInfo* ci, int ncol, int nq, double* out,
                  hipStream_t st);
int launch_finalize(const double* solve_partials, int nsolve, const double* col_sums,
                    const ColInfo* ci, int ncol, const double* ld_partials, int nld,
                    const double* yhat0, int64_t n, Params* P, const KDesc& kd, double* out3,
                    double* grad, double* tau_hat, hipStream_t st);

// ---- points.hip
int launch_gen_points(const uint32_t* gen, const uint32_t* shift, int family, int d, int m,
                      int64_t first, int64_t count, uint32_t* out, hipStream_t st);
struct PredTasks {
  int m[MTGP_MAXT];
  int64_t off[MTGP_MAXT];
};
// training points of the direct sum split into chunks of `chunk` indices;
// chunks [cstart[u], cstart[u+1]) belong to task u
struct PredChunks {
  int64_t chunk;
  int cstart[MTGP_MAXT + 1];
};
// part holds cstart[T] * M doubles of partial sums
template <typename Real>
int launch_predict_direct(const uint32_t* gen, const uint32_t* shifts, const PredTasks& pt,
                          const PredChunks& pc, const double* alpha, const uint32_t* xs,
                          int64_t M, const Params* P, const KDesc& kd, double* part, double* mean,
                          hipStream_t st);

// ---- lattice.hip (complex values interleaved re, im)
template <typename R>
struct alignas(2 * sizeof(R)) cx {
  R x, y;
};
enum { LAT_SRC_GEN = 0, LAT_SRC_Y = 1, LAT_SRC_X = 2 };  // columns, bit-reversed data, plain data
int launch_lat_natural(const void* spec, int spec_f32, void* X, int64_t nvec, int m,
                       hipStream_t st);
int lat_single_pass(int m);
template <typename R>
int launch_lat_single_natural(int src, const void* x, int x_f32, cx<R>* X, int nvec, int m,
                              hipStream_t st);
enum { LAT_SINK_Z = 0, LAT_SINK_REDUCE = 1, LAT_SINK_REAL = 2 };
int lat_adj_blocks(int m, size_t cbytes);
template <typename CR, typename SR>
int launch_lat_forward(int src, cx<CR>* work, cx<SR>* spec, int64_t vstride, int nvec, int m,
                       const void* y, int y_f32, double scale, const uint32_t* gen, const uint32_t* colshift,
                       const Params* P, const KDesc& kd, hipStream_t st, int natural = 0);
// Whether launch_lat_forward can write natural frequency order itself
// (natural = 1: a multi-pass length whose last pass is the wave pass).
int lat_natural_out(int m);
template <typename CR, typename SR>
int launch_lat_adjoint(int sink, const cx<SR>* spec, cx<CR>* work, double* real_out,
                       int64_t vstride, int nvec, int m, int conj_in, double scale,
                       const uint32_t* gen, const uint32_t* colshift, const Params* P,
                       const KDesc& kd, double* partials, hipStream_t st);

// ---- alg1.hip
constexpr int MTGP_MAXCOL = MTGP_MAXT + MTGP_MAXT * (MTGP_MAXT - 1) / 2;
struct z2 {
  double x, y;
};
struct Alg1Desc {
  int T, profile;
  int m[MTGP_MAXT];
  int64_t msz[MTGP_MAXT];        // block size after stage s: sum_{t<=s} n_t / n_s
  int64_t stage_off[MTGP_MAXT];  // offset of stage s in the log-pivot buffer
  int64_t task_off[MTGP_MAXT];   // offset of task t in yhat / ahat (elements)
  alignas(4) uint8_t pair_col[MTGP_MAXT][MTGP_MAXT];
  alignas(4) uint8_t diag_first[MTGP_MAXT];  // first task with the same length
  int col_m[MTGP_MAXCOL];
  int64_t col_off[MTGP_MAXCOL];
  // fill-free elimination: pattern row a (pairs (a, b >= a), n_a entries
  // each) starts at so[a], so[T] = total; class-0 node (t, k) (frequency
  // k n_T) sits at coff[t] + k of each of the T unit right-hand sides
  int64_t so[MTGP_MAXT + 1];
  int64_t coff[MTGP_MAXT];
  __host__ __device__ inline int pc(int t, int u) const { return u8_at(pair_col[t], u); }
  __host__ __device__ inline int df(int t) const { return u8_at(diag_first, t); }
};
constexpr int64_t ALG1_MAX_BLOCK = 2048;  // largest final block N / n_T handled
template <typename SR>
int launch_alg1(SR* cols, const Alg1Desc& A1, Params* P, int family, bool grad,
                const double* yhat, z2* bufA, z2* bufB, double* logs, double* ahat,
                double* partials, int* status, hipStream_t st);

// position of frequency f in a spectrum of length 2^m (digital sequences:
// natural order; lattices: bit-reversed order, the output order of the
// decimation-in-frequency transform)
__device__ inline int64_t spec_pos(int family, int64_t f, int m) {
  if (family == FAM_DSEQ || m == 0) return f;
  return (int64_t)(__brevll((unsigned long long)f) >> (64 - m));
}

// lambda of column c (log2 length m) at frequency f, as a complex number
template <typename SR>
__device__ inline z2 lam_at(const SR* cols, const Alg1Desc& A1, int family, int c, int64_t f) {
  const int m = A1.col_m[c];
  const int64_t pos = A1.col_off[c] + spec_pos(family, f, m);
  if (family == FAM_DSEQ) return {(double)cols[pos], 0.0};
  return {(double)cols[2 * pos], (double)cols[2 * pos + 1]};
}

// ---- elim.hip
// Workspace of the fill-free elimination (complex entries): pattern values
// so[T], the data right-hand side N, the unit right-hand sides T msz[T-1].
inline int64_t zf_elems(const Alg1Desc& A1, int64_t N) {
  return A1.so[A1.T] + N + (int64_t)A1.T * A1.msz[A1.T - 1];
}
constexpr int ZF_FINAL_BLOCKS = 2048;  // partial rows of the final pass (at most)
inline int64_t zf_final_blocks(int64_t N) {
  const int64_t b = (N + 255) / 256;
  return b < ZF_FINAL_BLOCKS ? b : ZF_FINAL_BLOCKS;
}
template <typename SR>
int launch_zerofill_gcv(SR* cols, const Alg1Desc& A1, int64_t N, Params* P, int family,
                        const double* yhat, z2* buf, double* logs, double* partials, int* status,
                        hipStream_t st);
template <typename SR>
int launch_zerofill(SR* cols, const Alg1Desc& A1, int64_t N, Params* P, int family, bool grad,
                    const double* yhat, z2* buf, double* logs, double* ahat, double* partials,
                    int* status, hipStream_t st);

// ---- elim_gcv.hip
// GCV at nested sizes in dual numbers (value, derivative under Lambda + e I):
// weights = false runs the elimination, the means and the (q, s) pass;
// weights = true writes the gradient weights (q, s in P).  buf holds
// zf_elems(A1, N) pairs of complex values.
template <typename SR>
int launch_zerofill_gcv_dual(SR* cols, const Alg1Desc& A1, int64_t N, Params* P, int family,
                             const double* yhat, void* buf, double* partials, int* status,
                             bool weights, hipStream_t st);

// ---- gcv.hip
template <typename SR>
int launch_gcv_eq(SR* cols, int64_t n, const PairMap& pm, const double* yhat, const Params* P,
                  const KDesc& kd, bool grad, double* partials, int* status, hipStream_t st);

// ---- cubature.hip
struct CubDesc {
  int equal;
  int64_t n;                            // equal sizes: common length
  uint8_t pair_col[MTGP_MAXT][MTGP_MAXT];  // column of pair (t <= u)
  int64_t task_off[MTGP_MAXT];          // task offsets in ahat
};
template <typename SR>
int launch_cubature(const SR* cols, const CubDesc& cd, const double* ahat, const Params* P,
                    const KDesc& kd, double* mu, double* Sigma, hipStream_t st);

// ---- postvar.hip
int launch_var_shifts(const uint32_t* xs, int64_t Mb, const uint32_t* taskshift, int T, int d,
                      int family, uint32_t* out, hipStream_t st);
template <typename SR>
int launch_var_eq(const SR* cols, int64_t n, const PairMap& pm, int family, const double* mu,
                  int64_t Mb, const Params* P, int T, double* partials, int nbx, hipStream_t st);
int launch_var_nested(const double* mu, const Alg1Desc& A, int family, int64_t N, int64_t Mb,
                      const Params* P, const z2* S, z2* Y, double* partials, int nbx,
                      hipStream_t st);
int launch_var_finalize(const double* partials, int nbx, int64_t Mb, int rowm, bool equal,
                        const Params* P, const KDesc& kd, double* var, hipStream_t st);
inline int var_tm(int T) { return T <= 1 ? 1 : T <= 2 ? 2 : T <= 4 ? 4 : T <= 8 ? 8 : 16; }

// ---- batch.hip
// One fit of a many-fit batch: its plan's tables and workspace regions, the
// caller's theta / outputs / Adam state, and its slice of the batch
// workspace (pattern storage of the fill-free elimination, log pivots, the
// solve's partial row, one adjoint row per column, the log-pivot sum).
struct BFit {
  KDesc kd;  // unequal = 1: every fit goes through the fill-free elimination
  Alg1Desc A;
  int ncol, sr_f32;
  int64_t N;
  const uint32_t* gen;
  const uint32_t* colshift;
  const ColInfo* colinfo;
  const double* theta;
  double* out3;
  double* grad;
  Params* P;
  int* status;
  void* cols;    // spectrum / adjoint weights (float when sr_f32, else double)
  double* work;  // FP64 working values (== cols for FP64 fits)
  double* yhat;
  z2* S;
  double* logs;
  double* sp;
  double* ap;
  double* m1;
  double* m2;
  int64_t* step;
  const uint8_t* frozen;
  int64_t ntheta;
};
struct BItem {
  int fit, col;
};
constexpr int BATCH_MAX_M = 14;  // per-task sizes of the many-fit path: n_t <= 2^14
constexpr int BATCH_SOLVE_BLOCKS = 64;  // workgroups per fit of each elimination launch
// launch groups of column items sharing a kernel type and dimension width
int launch_batch_prep(const BFit* fits, int nfits, hipStream_t st);
int launch_batch_fwd(const BFit* fits, const BItem* items, int nitems, int kt, int d,
                     hipStream_t st);
int launch_batch_solve(const BFit* fits, int nfits, int tmax, hipStream_t st);
int launch_batch_adj(const BFit* fits, const BItem* items, int nitems, int kt, int d,
                     hipStream_t st);
int launch_batch_final(const BFit* fits, int nfits, hipStream_t st);
int launch_batch_adam(const BFit* fits, int nfits, double lr, double b1, double b2, double eps,
                      hipStream_t st);

// ---- optim.hip
int launch_adam(double* theta, const double* grad, double* m1, double* m2, int64_t n, double lr,
                double b1, double b2, double eps, int64_t* step, const uint8_t* frozen,
                hipStream_t st);

// ---- prednet.hip
struct PredNet {
  int T, m_star;
  int m[MTGP_MAXT];
  int64_t col_off[MTGP_MAXT];   // test-net column of task u in the scratch buffer
  int64_t task_off[MTGP_MAXT];  // ahat of task u
};
int launch_prednet_shifts(const uint32_t* host_shifts, int count, uint32_t* dev, hipStream_t st);
int launch_prednet_fold(const double* lam, const PredNet& pn, const double* ahat, const Params* P,
                        double* w, hipStream_t st);
int launch_prednet_out(const double* w, const PredNet& pn, const Params* P, double* mean,
                       hipStream_t st);
int launch_prednet_lat_fold(const double* lam, const PredNet& pn, const double* ahat,
                            const Params* P, double* w, hipStream_t st);
int launch_prednet_lat_out(const double* ureal, const PredNet& pn, const Params* P, double* mean,
                           hipStream_t st);

}  // namespace mtgp

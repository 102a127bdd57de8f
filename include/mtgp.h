/*
 * mtgp.h -- C ABI of the MI355X (gfx950) fast multitask Gaussian-process
 * likelihood library.
 *
 * The library evaluates, exactly, the MLE loss of a multitask GP with the
 * product kernel K((t,x),(t',x')) = R_tt' Q(x,x') (Eq. mtprod), its gradient
 * and the posterior mean, on the design-kernel pairings of Condition
 * "Fast MTGP":
 *   MTGP_DSEQ: digitally shifted base-2 digital sequences in radical-inverse
 *              order (Def. "Base-2 digitally-shifted digital sequences") with
 *              digitally-shift-invariant kernels (Eq. DSI_kernel_1d_ex),
 *              diagonalised by the Walsh-Hadamard transform;
 *   MTGP_LAT:  shifted rank-1 lattices in radical-inverse order (Def.
 *              "Shifted rank-1 lattice") with shift-invariant Bernoulli kernels
 *              (Eq. SI_kernel_1d_ex), diagonalised by bit reversal + DFT.
 * Task t has n_t = 2^m_t points, n_1 >= ... >= n_T, a common generator and
 * its own shift; the Gram matrix factors as Ktilde = V Lambda V^dagger
 * (Theorem "Fast MTGP computations") and Lambda is inverted per frequency
 * (equal sizes) or, for nested unequal sizes, by elimination in task order:
 * by default as a fill-free sparse LDL^H factorisation (the task-order
 * pivots of Algorithm "Inverse and log-determinant of Lambda" without its
 * dense blocks), or by the algorithm as printed (mtgp_plan_set_elimination).
 *
 * Conventions for every entry point:
 *   - Pointers named `stream` are hipStream_t values passed as void*.
 *   - Device pointers: theta, y, out3, grad, tau_hat, mean, xs, cols, ws, x, X,
 *     out.  Host pointers: everything inside mtgp_design, and the arguments
 *     of mtgp_plan_create / mtgp_status / the query functions.
 *   - Calls that take a stream only enqueue work; none synchronises, none
 *     allocates device memory, so they may be captured in a HIP graph.
 *     Errors found on the device (a non-positive pivot, a NaN) are written to
 *     a status word inside `ws` and read back with mtgp_status after the
 *     caller synchronises.
 *   - The caller owns every buffer.  `ws` is a device buffer of
 *     mtgp_workspace_bytes(plan) bytes; it holds the transformed data written
 *     by mtgp_set_data and scratch for the other calls, so calls that share a
 *     `ws` must be ordered on one stream.
 *   - Threads.  The compute calls (mtgp_kernel_cols .. mtgp_cubature) do not
 *     change a plan, except for the overlap fork of digital-net plans: the
 *     plan's own stream and a ring of events, taken under a lock inside the
 *     plan.  So several host threads may issue compute calls on one plan at
 *     once, each with its own `ws` and stream; their overlapped high passes
 *     then queue one after the other on the plan's stream (correct, but not
 *     concurrent).  The configuration calls (mtgp_plan_set_*, enable_timing,
 *     destroy) and mtgp_phase_times must not run concurrently with any other
 *     call on the same plan, and phase timing records into the plan, so a
 *     timed plan must be used from one thread.
 *   - Return value: MTGP_OK or a negative MTGP_E* code (see mtgp_strerror).
 *
 * Hyperparameter vector theta (FP64, device), packed in this order:
 *   tau[T] | log gamma | log eta[d] | log b[4] (adaptive DSI kernels only) |
 *   log xi[T] | B[T][s] (row-major) | log zeta[T]
 * with R = B B^T + diag(zeta) (Section "Multitask Setting"), Q(x,x') =
 * gamma prod_j [1 + eta_j K(x_j,x'_j)] (Eq. prod_kernel), K = Khat_order or
 * sum_alpha b_alpha Khat_alpha (adaptive), and per-task noise xi_t.
 * The gradient is returned in the same packing, with respect to the packed
 * coordinates (log-parameters where the packing says log).
 * Data y (FP64, device, length N = sum n_t) is task-major, each task in the
 * radical-inverse order of its points (i = 0 .. n_t - 1).
 * Points and test inputs are 32-bit digits u standing for x = u 2^-32.
 */
#ifndef MTGP_H
#define MTGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MTGP_OK = 0,
  MTGP_EINVAL = -1,   /* invalid argument (sizes, ordering, null pointer, order) */
  MTGP_ENOTPD = -2,   /* Lambda not positive definite at some frequency / NaN */
  MTGP_EHIP = -3,     /* a HIP runtime call failed */
  MTGP_ENOMEM = -4,   /* plan creation could not allocate its small tables */
  MTGP_ENOTSUP = -5,  /* combination not supported by this build */
  MTGP_ETOOBIG = -6   /* input exceeds the static scratch of an allocation-free entry point */
};

enum { MTGP_DSEQ = 0, MTGP_LAT = 1 };
/* Precision modes.  Per-frequency factorisations, log-det and quadratic-form
 * reductions are FP64 in all of them.
 *   MTGP_FP64:  everything FP64.
 *   MTGP_MIXED: all arithmetic FP64 (kernel columns, transforms, adjoint,
 *               derivative reduction); only the finished spectrum, the
 *               adjoint weights and (equal sizes) the copy of the data
 *               transform that the per-frequency solves read are stored in
 *               FP32 (a relative rounding per entry; frequency 0 is read in
 *               FP64), which halves the bytes of the solve and of the last
 *               forward / first adjoint transform pass.  FP32 arithmetic in
 *               the columns or transforms was measured to make Lambda
 *               indefinite on the T=8, d=10, n=2^24 net design (the
 *               transform's absolute rounding ~eps32 ||c||_2 exceeds the
 *               noise variance), and FP32 element sums in the adjoint moved
 *               the gradient by 6.8%, so neither is used here.
 *   MTGP_F32:   kernel columns and all transform arithmetic in FP32.  The
 *               transform's absolute rounding error (~eps32 ||c||_2 sqrt(m))
 *               exceeds small noise variances xi at large n, which makes
 *               Lambda indefinite (reported as MTGP_ENOTPD); kept to measure
 *               exactly that. */
enum { MTGP_FP64 = 0, MTGP_MIXED = 1, MTGP_F32 = 2 };
enum { MTGP_DTYPE_F64 = 0, MTGP_DTYPE_F32 = 1 };
/* Elimination for nested unequal sizes (mtgp_plan_set_elimination). */
enum { MTGP_ELIM_SPARSE = 0, MTGP_ELIM_ALG1 = 1 };

typedef struct mtgp_plan mtgp_plan;

typedef struct mtgp_design {
  int32_t T;             /* number of tasks, 1 <= T <= 16 */
  int32_t d;             /* input dimension, 1 <= d <= 32 */
  int32_t family;        /* MTGP_DSEQ or MTGP_LAT */
  const int32_t* m;      /* [T] log2 sizes, non-increasing (Condition "Fast MTGP"), 0 <= m_t <= 30 */
  const uint32_t* gen;   /* DSEQ: [d][32] generating columns, column p = image of input digit p
                            (bit 31 is the first output digit); LAT: [d] odd generating vector */
  const uint32_t* shift; /* [T][d] digital shift (DSEQ) or lattice shift times 2^32 (LAT) */
  int32_t kernel_order;  /* DSI: 1..4; SI: 1..3 (alpha of the Bernoulli polynomial B_{2 alpha}) */
  int32_t adaptive;      /* DSI only: K = sum_{alpha=1..4} b_alpha Khat_alpha with weights in theta */
  int32_t rank_s;        /* number of columns of B, 1 <= s <= 16 */
  int32_t profile_tau;   /* 1: tau = tau_hat_MLE (Eq. MTGP_optimal_tau), theta's tau ignored and its
                            gradient zero; 0: tau taken from theta */
} mtgp_design;

/* Validates the design, copies it, and uploads its small tables (generating
 * matrices, shifts, column schedule) to the current HIP device.  Errors:
 * MTGP_EINVAL (T, d, m ordering, m > 30, even lattice generator, unsupported
 * order, adaptive with LAT), MTGP_ENOMEM, MTGP_EHIP. */
int mtgp_plan_create(const mtgp_design* design, int32_t precision, mtgp_plan** out);
int mtgp_plan_destroy(mtgp_plan* plan);

/* Transform schedule (tuning only; results are the same up to rounding):
 * each length-2^m transform runs as one LDS-resident pass over the low
 * pass_a_bits index bits (1..13; fused with kernel-column generation) and
 * passes over at most pass_b_bits (1..12) further bits each, or, with
 * pass_b_bits = 0, by size: the whole remainder in one pass when it is 8, 10
 * or 12 bits (and the one-pass kernel takes it), else passes of at most 6
 * bits.  Passes of at most 6 bits above bit 8 keep each thread's 2^bits
 * strided values in registers.  Passes of exactly 8 or 10 bits (above bit
 * 8 - bits/2, with a block's window below 2^30 bytes) go through registers
 * and one LDS tile of 256 x 2^(bits/2) values.  A 12-bit pass (above bit 3)
 * holds 4096 rows of 2, 4 or 8 adjacent columns in registers, the widest
 * whose exchange grid of 8.6 KiB per column (FP64; half in FP32) fits
 * pass_b_tile_bytes, and transposes them through that grid in four
 * quarter-size rounds.  Other wider passes use an LDS tile of about
 * pass_b_tile_bytes (4096..147456).  Changes mtgp_workspace_bytes, so call
 * it before sizing the workspace.  Defaults: 12, 0, 73728 (measured on
 * MI355X: at 2^24-point columns the 12 high bits in one pass of 8 columns
 * per block, 11.7 -> 10.2 ms per loss + gradient at T=8, d=10 with the
 * passes in sequence). */
int mtgp_plan_set_schedule(mtgp_plan* plan, int32_t pass_a_bits, int32_t pass_b_bits,
                           int64_t pass_b_tile_bytes);

/* Elimination used by nested unequal sizes (ignored for equal sizes; both
 * eliminate the tasks in order with the same pivots, so results agree up to
 * rounding):
 *   MTGP_ELIM_SPARSE (default): Lambda = L D L^H with L on Lambda's own
 *     pattern (task-order elimination creates no fill because the later
 *     neighbours of a node (t, f), the nodes (u, f mod n_u), u > t, are
 *     coupled to each other); O(N T^2) work and sum_t (T - t) n_t stored
 *     entries, with Lambda^-1 on the pattern from the factor for the gradient.
 *   MTGP_ELIM_ALG1: Algorithm "Inverse and log-determinant of Lambda" with
 *     dense running-inverse blocks of size m_T = sum_t n_t / n_T (requires
 *     m_T <= 2048, else MTGP_ENOTSUP; two buffers of N m_T complex values).
 * Changes mtgp_workspace_bytes, so call it before sizing the workspace.
 * Errors: MTGP_EINVAL (mode), MTGP_ENOTSUP. */
int mtgp_plan_set_elimination(mtgp_plan* plan, int32_t mode);

/* Digital nets: at most blocks_per_cu workgroups per compute unit of the
 * fused column-generation and derivative-reduction kernels (1..8; 0, the
 * default: as many as fit), enforced through their LDS request.  With the
 * overlapped passes (mtgp_plan_set_overlap) a cap leaves room on each
 * compute unit for the HBM-bound strided passes running beside them.  A
 * schedule parameter: results are bitwise the same.  Errors: MTGP_EINVAL. */
int mtgp_plan_set_fused_occupancy(mtgp_plan* plan, int32_t blocks_per_cu);

/* Overlap of the digital-net passes (tuning only; results are bitwise the
 * same): the columns of each length group are processed in `chunks` chunks
 * (1..32, at most the group's column count; default 4).  The VALU-bound fused passes (generation + low
 * transform bits, adjoint low bits + derivative reduction) run on the
 * caller's stream and the HBM-bound high transform passes on a stream owned
 * by the plan, forked from and joined back into the caller's stream through
 * events.  chunks = 1 runs every pass on the caller's stream in order, and
 * so does every call made while the caller's stream is being captured into
 * a HIP graph.  Lattice plans ignore it. */
int mtgp_plan_set_overlap(mtgp_plan* plan, int32_t chunks);

/* Profiling aid (not thread safe): when enabled, every loss evaluation of the
 * plan (mtgp_nll, mtgp_nll_grad and the loss inside mtgp_predict*) records
 * HIP events on the caller's stream between its phases, into a ring of 64
 * event sets, so consecutive calls are timed without any host wait.
 * mtgp_phase_times waits for the last recorded event and writes to
 * ms[0 .. max_phases-1] the mean duration in ms of each phase over the calls
 * recorded since the previous mtgp_phase_times (or since enabling; the 64 most
 * recent if more), then starts a new count; all zero if none was recorded.
 * *nphases receives the number of phases, mtgp_phase_name(k) their names:
 * prep, gen_fwd_low (column generation fused with the low-bit transform
 * pass), fwd_high, solve, adj_high, adj_low_reduce (adjoint low-bit pass
 * fused with the derivative reduction), finalize (partial-sum reductions and
 * the chain rule).  Enabling or disabling resets the count. */
int mtgp_plan_enable_timing(mtgp_plan* plan, int32_t on);
int mtgp_phase_times(const mtgp_plan* plan, double* ms, int32_t max_phases, int32_t* nphases);
const char* mtgp_phase_name(int32_t k);

/* Number of FP64 entries of theta (and of the gradient). */
int64_t mtgp_theta_size(const mtgp_plan* plan);
/* Bytes of the device workspace `ws` the other calls need. */
size_t mtgp_workspace_bytes(const mtgp_plan* plan);
/* Total number of data points N = sum_t n_t. */
int64_t mtgp_num_points(const mtgp_plan* plan);
/* Distinct kernel columns (Theorem "Fast MTGP computations", item 3: one
 * zeroth column per task pair, tall case; pairs with equal length and equal
 * pair shift share a column, e.g. all diagonal pairs of equal-size tasks).
 * mtgp_column_info reports column c's log2 length, its offset (in elements)
 * inside the buffer written by mtgp_kernel_cols, and one task pair (t <= u)
 * that uses it. */
int32_t mtgp_num_columns(const mtgp_plan* plan);
int mtgp_column_info(const mtgp_plan* plan, int32_t c, int32_t* log2n, int64_t* offset,
                     int32_t* t, int32_t* u);

/* Points x_{t,i}, i = first .. first+count-1, of task t (0-based) as digits,
 * out[count][d] (Def. "Base-2 digitally-shifted digital sequences":
 * x_i = (XOR_{p: i_p = 1} g_p) XOR Delta_t; Def. "Shifted rank-1 lattice":
 * x_i = (v(i) g + Delta_t) mod 1).  Bit-exact.  Indices may exceed n_t (the
 * sequences are extensible) but must stay below 2^32. */
int mtgp_gen_points(const mtgp_plan* plan, int32_t task, int64_t first, int64_t count,
                    uint32_t* out, void* stream);

/* Raw kernel columns c_p(i) = Q(z_i XOR s_p) (DSEQ, i in radical-inverse
 * order) or Q((j g / n + s_p) mod 1) (LAT, natural lattice order j), one per
 * distinct column, without the task factor R, in the plan's column precision
 * (FP64 and MIXED plans: double, F32 plan: float).  `cols` holds
 * sum_c 2^log2n(c) elements laid out at the offsets of mtgp_column_info.
 * (Eq. prod_kernel; Theorem "Fast MTGP computations", item 3.) */
int mtgp_kernel_cols(const mtgp_plan* plan, const double* theta, void* cols, void* ws,
                     void* stream);

/* In-place unnormalised Walsh-Hadamard transform of `batch` contiguous
 * vectors of length 2^log2n, natural (Sylvester) order:
 * X_f = sum_i (-1)^popcount(f & i) x_i  (the V^dagger of Theorem "Fast GP
 * computations" for DSEQ, up to the factor 2^(-log2n/2)).  dtype is
 * MTGP_DTYPE_F64 or MTGP_DTYPE_F32; 0 <= log2n <= 30; batch 0 does nothing
 * (x may then be NULL). */
int mtgp_fwht(void* x, int64_t batch, int32_t log2n, int32_t dtype, void* stream);

/* Unnormalised forward DFT X_f = sum_j x_j e^{-2 pi i f j / n} of `batch`
 * contiguous real vectors of length n = 2^log2n into complex outputs in
 * natural frequency order (interleaved re, im; X has batch * n complex
 * entries).  If bitrev_input is nonzero the input is first read in
 * bit-reversed order, i.e. the transform is the V^dagger of Theorem "Fast GP
 * computations" for lattices times sqrt(n).  dtype as for mtgp_fwht;
 * 0 <= log2n <= 30, batch <= 65535.  For log2n > 12 the multi-pass transform
 * needs `scratch` with room for batch * n complex values of dtype (else it
 * may be NULL); scratch and X must not overlap.  batch 0 does nothing (the
 * pointers may then be NULL). */
int mtgp_fft(const void* x, void* X, void* scratch, int64_t batch, int32_t log2n, int32_t dtype,
             int32_t bitrev_input, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mtgp_fft
 * without the scratch argument.  Same transform, arguments and results as
 * mtgp_fft.  The multi-pass sizes (log2n > 12) stage the bit-reversed
 * spectrum in a static device array of MTGP_FFT_NOALLOC_SCRATCH_BYTES bytes
 * (32 MiB) that each GPU the library runs on holds until the process ends;
 * batch * 2^log2n complex values of dtype (16 B for F64, 8 B for F32) must
 * fit in it, else MTGP_ETOOBIG and nothing is enqueued.  The call allocates
 * nothing: the array's device address is looked up once per device, on that
 * device's first call (hipGetSymbolAddress; MTGP_EHIP if that fails), so
 * make one call outside any capture before capturing.  Every call on a GPU
 * shares that GPU's array, and every entry of it is written before it is
 * read, so nothing carries over between calls; calls that overlap in time on
 * one GPU (two streams, two threads) race on it and must be ordered by the
 * caller. */
#define MTGP_FFT_NOALLOC_SCRATCH_BYTES 33554432
int mtgp_fft_noalloc(const void* x, void* X, int64_t batch, int32_t log2n, int32_t dtype,
                     int32_t bitrev_input, void* stream);

/* Transforms the data once per data set: yhat_t = V^dagger_{m_t} y_t
 * (Theorem "Fast MTGP computations"), kept inside ws for later calls. */
int mtgp_set_data(const mtgp_plan* plan, const double* y, void* ws, void* stream);

/* MLE loss (Eq. MTGP_MLE_GCV_loss): out3[0] = (y - E^T tau)^T Ktilde^-1 (y - E^T tau),
 * out3[1] = log det Ktilde, out3[2] = their sum L.  tau_hat (may be NULL)
 * receives the means used (tau_hat_MLE when profiling, Eq. MTGP_optimal_tau;
 * theta's tau otherwise).  Requires mtgp_set_data on the same ws. */
int mtgp_nll(const mtgp_plan* plan, const double* theta, double* out3, double* tau_hat, void* ws,
             void* stream);

/* As mtgp_nll, plus grad = dL/dtheta in the packed coordinates.  The paper
 * gives no gradient formula; this is the exact derivative of L (adjoint of
 * Ktilde = V Lambda V^dagger with V independent of theta). */
int mtgp_nll_grad(const mtgp_plan* plan, const double* theta, double* out3, double* grad,
                  double* tau_hat, void* ws, void* stream);

/* Posterior mean (Eq. MTGP_post_mean_cov) at M arbitrary inputs xs[M][d]
 * (digits): mean[M][T], mean[m][t] = tau_t + sum_t' R_tt' sum_k
 * Q(x*_m, x_t'k) alpha_t'k with alpha = Ktilde^-1 (y - E^T tau).  Direct
 * sum, O(M N d).  Requires mtgp_set_data.  M = 0 does nothing. */
int mtgp_predict(const mtgp_plan* plan, const double* theta, const uint32_t* xs, int64_t M,
                 double* mean, void* ws, void* stream);

/* Posterior mean on a structured test net: the first 2^m_star points of the
 * plan's sequence with shift shift_star[d] (host; a digital shift for nets,
 * a lattice shift times 2^32 for lattices), in radical-inverse order:
 * mean[2^m_star][T].  Uses the cross-block structure of Theorem "Fast MTGP
 * computations" for each (test net, task) pair (for lattices: a cyclic
 * convolution on the finer of the two lattices, folded onto the test
 * frequencies), O(N log N + T n* log n*) instead of O(M N d).  `scratch` is
 * a device buffer of mtgp_predict_net_scratch_bytes(plan, m_star) bytes.  Requires
 * mtgp_set_data; 0 <= m_star <= 30. */
size_t mtgp_predict_net_scratch_bytes(const mtgp_plan* plan, int32_t m_star);
int mtgp_predict_net(const mtgp_plan* plan, const double* theta, const uint32_t* shift_star,
                     int32_t m_star, double* mean, void* ws, void* scratch, void* stream);

/* Posterior variance (Eq. MTGP_post_mean_cov, the covariance at (t, x) =
 * (t', x')) at M arbitrary inputs xs[M][d] (digits): var[M][T],
 *   var[m][t] = R_tt Q(x_m, x_m) - k(t, x_m)^T Ktilde^-1 k(t, x_m),
 *   k(t, x) = (R_tu Q(x, x_uk))_{u, k}  (the latent f, without noise).
 * Per test point the T cross columns Q(x, x_uk) are generated and
 * transformed like kernel columns (Theorem "Fast MTGP computations":
 * V^dagger k has blocks R_tu V_u^dagger Q(x, x_u.)), and the quadratic form
 * runs through the loss's factorisation: per-frequency L D L^H at equal
 * sizes, forward substitution through the fill-free task-order factor at
 * nested sizes (MTGP_ELIM_SPARSE; MTGP_ELIM_ALG1 returns MTGP_ENOTSUP).
 * O(N log N + N T^2) per test point.  Test points are processed `batch` at
 * a time in `scratch`, a device buffer of
 * mtgp_predict_var_scratch_bytes(plan, batch) bytes.  Runs one loss
 * evaluation on ws (data set by mtgp_set_data).  The result is a difference
 * of two terms of size R_tt Q(x, x): its rounding is relative to that scale,
 * not to var.  M = 0 does nothing. */
size_t mtgp_predict_var_scratch_bytes(const mtgp_plan* plan, int32_t batch);
int mtgp_predict_var(const mtgp_plan* plan, const double* theta, const uint32_t* xs, int64_t M,
                     int32_t batch, double* var, void* ws, void* scratch, void* stream);

/* GCV loss (Eq. MTGP_MLE_GCV_loss): out3 = (q, s, L_GCV) with
 * q = r^T Ktilde^-2 r, s = tr Ktilde^-1, L_GCV = q / s^2, r = y - E^T tau,
 * and optionally its gradient (device [theta size], same packing as
 * mtgp_nll_grad; NULL: loss only).  tau is the plan's fixed means or, when
 * profiled, the optimal GCV means (Eq. MTGP_optimal_tau), which for equal
 * sizes are the per-task sample means (written to tau_hat if non-NULL).
 * Equal sizes: two passes over the spectrum (q and s first).  Nested sizes
 * (MTGP_ELIM_SPARSE only; Algorithm 1's elimination returns MTGP_ENOTSUP):
 * the loss and means through the fill-free elimination, s from the diagonal
 * of its selected inverse; the gradient runs that elimination in dual
 * numbers under Lambda + e I, whose derivative parts are -Lambda^-2 on
 * Lambda's pattern and -Lambda^-2 rhat, then a pass for q and s and one for
 * the weights W = -(b a^H + a b^H) / s^2 + (2 q / s^3) Lambda^-2.
 * Same workspace as mtgp_nll_grad. */
int mtgp_gcv(const mtgp_plan* plan, const double* theta, double* out3, double* grad,
             double* tau_hat, void* ws, void* stream);

/* Multitask Bayesian cubature (Section "Extensions for Bayesian Cubature",
 * multitask theorem): the posterior N(mu_hat, Sigma) of the task integrals
 * mu_t = int_[0,1)^d f(t, x) dx under the fitted MTGP,
 *   mu_hat = tau + gamma R E Ktilde^-1 (y - E^T tau)   (device [T]),
 *   Sigma  = gamma R - gamma^2 R Pi R, Pi = E Ktilde^-1 E^T   (device [T][T]),
 * with tau the plan's means (profiled: mu_hat = tau_hat).  Runs one loss
 * evaluation on ws (data set by mtgp_set_data) plus an O(T^3) kernel. */
int mtgp_cubature(const mtgp_plan* plan, const double* theta, double* mu_hat, double* Sigma,
                  void* ws, void* stream);

/* Many independent fits: mtgp_nll_grad for fit i = 0 .. nfits-1 with its own
 * plan, theta, outputs and workspace, all enqueued on one stream (host
 * arrays of device pointers).  Calls into it may be captured once in a HIP
 * graph and replayed (the library never synchronises or allocates), which
 * removes the per-launch host cost of many small fits. */
int mtgp_nll_grad_batched(int32_t nfits, mtgp_plan* const* plans, const double* const* thetas,
                          double* const* out3, double* const* grads, void* const* ws,
                          void* stream);

/* Many small independent fits with one launch per phase over all of them
 * (batching of the fitting loop; each fit is the loss and gradient of
 * mtgp_nll_grad for its own plan: Eq. MTGP_MLE_GCV_loss, Theorem "Fast MTGP
 * computations").  Phases: parameters; every kernel column of every fit
 * generated and transformed through all its index bits by one workgroup
 * (Walsh-Hadamard for nets, decimation in frequency for lattices); one
 * workgroup per fit for the elimination in task order (the fill-free
 * factorisation of the nested-size path, which equal sizes also take),
 * its selected inverse and the adjoint weights; the adjoint transform and
 * derivative sums per column; the chain rule per fit; optionally Adam.
 * Column phases are launched once per kernel type and padded dimension
 * width present in the batch.  Plans may differ in family, T, d, sizes
 * and kernel; each needs 2^m_1 <= 2^14 points per task and precision
 * MTGP_FP64 or MTGP_MIXED (else MTGP_ENOTSUP), mtgp_set_data on its own
 * `ws` beforehand, and the per-fit buffers below (host arrays of device
 * pointers, fixed at creation so the calls can be captured in a HIP graph
 * and replayed):
 *   ws[i]       the fit's workspace (mtgp_workspace_bytes of its plan);
 *   thetas[i]   theta, read by mtgp_batch_nll_grad, updated by Adam;
 *   out3[i], grads[i]  outputs as for mtgp_nll_grad;
 *   adam_m1/m2[i], adam_step[i]  Adam moments (zero before the first
 *               step) and device step counter, or adam_m1 = NULL for no
 *               Adam; frozen[i] as for mtgp_adam_step (frozen may be NULL);
 *   bws         device buffer of mtgp_batch_workspace_bytes(nfits, plans).
 * The batch keeps the plans' device tables: destroy it before them.
 * Creation allocates two small device tables; the compute calls allocate
 * nothing and never synchronise.  A batch must be used from one stream at
 * a time. */
typedef struct mtgp_batch mtgp_batch;
size_t mtgp_batch_workspace_bytes(int32_t nfits, mtgp_plan* const* plans);
int mtgp_batch_create(int32_t nfits, mtgp_plan* const* plans, void* const* ws,
                      double* const* thetas, double* const* out3, double* const* grads,
                      double* const* adam_m1, double* const* adam_m2, int64_t* const* adam_step,
                      const uint8_t* const* frozen, void* bws, mtgp_batch** out);
int mtgp_batch_destroy(mtgp_batch* batch);
int mtgp_batch_nll_grad(const mtgp_batch* batch, void* stream);
int mtgp_batch_adam_step(const mtgp_batch* batch, double lr, double beta1, double beta2,
                         double eps, void* stream);

/* One Adam step on the packed theta (device, length n <= 4096) with moments
 * m1, m2 (device, zero before the first step) and a device step counter
 * (int64, incremented by the call); entries with frozen[i] != 0 (device, may
 * be NULL) are left unchanged.  Graph-capturable. */
int mtgp_adam_step(double* theta, const double* grad, double* m1, double* m2, int64_t n, double lr,
                   double beta1, double beta2, double eps, int64_t* step, const uint8_t* frozen,
                   void* stream);

/* Reads the device status word of ws (synchronously, after the caller has
 * synchronised the stream).  Returns MTGP_OK or MTGP_ENOTPD; *bad_index (may
 * be NULL) receives the first frequency (or residue class) whose pivot was
 * not positive or not finite, else -1.  The status is cleared by
 * mtgp_set_data and at the start of every call that evaluates the loss
 * (mtgp_nll, mtgp_nll_grad, mtgp_predict with M > 0, mtgp_predict_net,
 * mtgp_gcv, mtgp_cubature). */
int mtgp_status(const mtgp_plan* plan, const void* ws, int64_t* bad_index);

const char* mtgp_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* MTGP_H */
